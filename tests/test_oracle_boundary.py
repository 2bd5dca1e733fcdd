"""Pins of the oracle's non-periodic boundaries: slip walls and characteristic
inflow/outflow, the conditions of the double Mach reflection and the jet
(Sec. 3.6).

- A slip wall is a mirror: a walled run equals, to rounding, the periodic run on
  the domain doubled across the wall with the data reflected (normal velocity
  negated), compared on the original half; for every limiter.
- Supersonic inflow imposes the exterior state: a run with inflow on x- equals
  the periodic run on a domain extended by a buffer holding the exterior state,
  on the elements the other boundary cannot reach in the steps taken.
- A closed box conserves mass and energy, keeps the positivity bounds on a blast
  that hits its walls, and keeps a state at rest.
- Every condition keeps a uniform flow whose exterior state is that flow
  (free-stream preservation), for sub- and supersonic speeds.
The subsonic characteristic branches are pinned by free-stream preservation
only; their values are checked against the rule they follow."""
import numpy as np
import pytest

from parity import state_err
from workloads import states
from workloads.meshes import MeshSpec, random_mesh, refined_box_mesh

G = 1.4


def _mirror(spec, axis):
    """The mesh doubled across the low wall of the axis: the original leaves
    moved to the upper half (first, in their order), their mirror images in the
    lower half."""
    lv = spec.level.astype(np.int64)
    if axis == 1:
        ny = spec.ny0 << lv
        ix = np.concatenate([spec.ix, spec.ix])
        iy = np.concatenate([spec.iy + ny, ny - 1 - spec.iy])
        return MeshSpec(np.concatenate([spec.level, spec.level]), ix.astype(np.int32),
                        iy.astype(np.int32), spec.x0, spec.y0 - spec.Ly, spec.Lx, 2 * spec.Ly,
                        spec.nx0, 2 * spec.ny0)
    nx = spec.nx0 << lv
    ix = np.concatenate([spec.ix + nx, nx - 1 - spec.ix])
    iy = np.concatenate([spec.iy, spec.iy])
    return MeshSpec(np.concatenate([spec.level, spec.level]), ix.astype(np.int32),
                    iy.astype(np.int32), spec.x0 - spec.Lx, spec.y0, 2 * spec.Lx, spec.Ly,
                    2 * spec.nx0, spec.ny0)


def _reflect(u, axis):
    """Mirror image of element states [E, 4, n, n] (e, v, b, a) across the axis."""
    r = u[:, :, ::-1, :] if axis == 1 else u[:, :, :, ::-1]
    r = r.copy()
    r[:, 1 + axis] *= -1.0
    return r


@pytest.mark.parametrize("limiter", ["positivity", "local", "combined"])
@pytest.mark.parametrize("axis", [0, 1])
def test_wall_is_a_mirror(oracle, axis, limiter):
    lim = {"positivity": oracle.LIM_POSITIVITY, "local": oracle.LIM_LOCAL,
           "combined": oracle.LIM_COMBINED}[limiter]
    spec = random_mesh(10, 6, 2, 0.4, L=2.0, x0=-1.0, y0=-1.0)
    bc = [0, 0, 1, 1] if axis == 1 else [1, 1, 0, 0]
    W = oracle.Mesh(3, *spec.args(), bc=bc)
    D = oracle.Mesh(3, *_mirror(spec, axis).args())
    assert W.NB > 0 and W.M > 0
    x, y, m = W.geometry()
    # a blast centred 0.35 from the low wall, with a shear flow on top
    c = (x + 0.65, y) if axis == 0 else (x, y + 0.65)
    r2 = c[0] ** 2 + c[1] ** 2
    u = states.conservative(1.0 + 0.2 * np.cos(np.pi * x) * np.sin(np.pi * y),
                            0.2 * np.sin(np.pi * y), 0.1 * np.cos(np.pi * x),
                            np.where(r2 <= 0.09, 3.0, 1e-3), G)
    d = np.concatenate([u, _reflect(u, axis)])
    E = W.E
    for _ in range(3):
        dt = W.max_dt(u, 0.5)
        assert abs(D.max_dt(d, 0.5) - dt) <= 1e-12 * dt
        u, sw = W.ssprk3_dt(u, dt, limiter=lim)
        d, sd = D.ssprk3_dt(d, dt, limiter=lim)
        assert sw["violations"] == 0
    err = state_err(u, d[:E])
    sym = state_err(d[:E], _reflect(d[E:], axis))
    print(f"wall axis {axis} {limiter}: walled vs mirrored {err:.2e}, mirror symmetry {sym:.2e}")
    tol = 1e-12 if limiter == "positivity" else 1e-9
    assert err < tol and sym < tol


def test_supersonic_inflow_is_the_exterior_state(oracle):
    """One limited forward-Euler step with characteristic inflow on x- equals the
    step on the domain extended by a buffer that holds the exterior state, on
    every element that x+ does not touch.  (Over several stages the LLF flux
    lets the buffer's upstream end react to the domain, so the equivalence is
    one stage long.)"""
    ext_prim = (1.2, 3.0, 0.1, 0.9)
    ext = states.conservative(*[np.array([q]) for q in ext_prim], G)[0]
    A = refined_box_mesh(8, (0.25, 0.25), (0.75, 0.75), 0.0, 0.0, 1.0)
    CH = oracle.BC_CHARACTERISTIC
    MA = oracle.Mesh(3, *A.args(), bc=[CH, CH, 0, 0], ext=np.tile(ext, (4, 1)))
    # the same leaves on [0, 2] x [0, 1], the right half a level-0 buffer
    bi, bj = np.meshgrid(np.arange(8, 16), np.arange(8), indexing="ij")
    B = MeshSpec(np.concatenate([A.level, np.zeros(64, np.int8)]),
                 np.concatenate([A.ix, bi.ravel()]).astype(np.int32),
                 np.concatenate([A.iy, bj.ravel()]).astype(np.int32), 0.0, 0.0, 2.0, 1.0, 16, 8)
    MB = oracle.Mesh(3, *B.args())
    x, y, m = MA.geometry()
    rho = 1.0 + 0.3 * np.exp(-((x - 0.05) ** 2 + (y - 0.5) ** 2) / 0.01)
    u = states.conservative(rho, 3.0 + 0 * x, 0.2 * np.sin(2 * np.pi * y), 1.0 + 0 * x, G)
    ub = np.concatenate([u, np.broadcast_to(ext[None, :, None, None], (64, 4, 4, 4))])
    assert 3.0 > np.sqrt(G / rho.min()) and ext_prim[1] > np.sqrt(G * ext_prim[3] / ext_prim[0])
    MO = oracle.Mesh(3, *A.args(), bc=[3, 3, 0, 0])
    dt = MA.max_dt(u, 0.9)
    near = x.max(axis=(1, 2)) <= 0.875
    left = x.min(axis=(1, 2)) == 0.0
    for lim in (oracle.LIM_NONE, oracle.LIM_POSITIVITY, oracle.LIM_LOCAL):
        a, _ = MA.fe_step(u, dt, limiter=lim)
        b, _ = MB.fe_step(ub, dt, limiter=lim)
        o, _ = MO.fe_step(u, dt, limiter=lim)
        err = state_err(a[near], b[: MA.E][near])
        act = state_err(a[left], o[left])
        print(f"supersonic inflow (limiter {lim}) vs buffer {err:.2e}; vs outflow {act:.2e}")
        assert err < 1e-14
        assert act > 1e-3  # the inflow acts


@pytest.mark.parametrize("limiter", ["positivity", "local"])
def test_closed_box_blast(oracle, limiter):
    lim = oracle.LIM_POSITIVITY if limiter == "positivity" else oracle.LIM_LOCAL
    spec = random_mesh(4, 6, 2, 0.4, L=1.0, x0=-0.5, y0=-0.5)
    M = oracle.Mesh(3, *spec.args(), bc=[1, 1, 1, 1])
    x, y, m = M.geometry()
    u = states.sedov_tophat(x - 0.1, y + 0.3, r0=0.15)
    tot0 = (u * m[:, None]).sum(axis=(0, 2, 3))
    for _ in range(8):
        u, st = M.ssprk3(u, 0.5, limiter=lim)
        assert st["violations"] == 0 and st["fv_inadmissible"] == 0
    tot = (u * m[:, None]).sum(axis=(0, 2, 3))
    scale = (np.abs(u) * m[:, None]).sum(axis=(0, 2, 3))
    rel = np.abs(tot - tot0) / scale
    print(f"closed box {limiter}: mass {rel[0]:.1e} energy {rel[3]:.1e} "
          f"momentum {rel[1]:.1e} {rel[2]:.1e}")
    assert rel[0] < 1e-13 and rel[3] < 1e-13
    # the wall pushes back: the blast, off centre, has gained momentum
    assert rel[1] > 1e-6 or rel[2] > 1e-6
    assert u[:, 0].min() > 0


def test_closed_box_rest_state(oracle):
    spec = random_mesh(4, 6, 2, 0.4)
    M = oracle.Mesh(4, *spec.args(), bc=[1, 1, 1, 1])
    x, y, m = M.geometry()
    u0 = states.constant(x, rho=1.3, v1=0.0, v2=0.0, p=0.8)
    for lim in (oracle.LIM_POSITIVITY, oracle.LIM_LOCAL):
        u = u0
        for _ in range(3):
            u, st = M.ssprk3(u, 0.9, limiter=lim)
        assert state_err(u, u0) < 1e-13


@pytest.mark.parametrize("kind", ["characteristic", "outflow", "wall-tangential"])
@pytest.mark.parametrize("speed", [0.4, 2.5])
def test_free_stream(oracle, kind, speed):
    spec = random_mesh(6, 6, 2, 0.4)
    if kind == "wall-tangential":  # flow along x with walls on y
        bc, v = [0, 0, 1, 1], (speed, 0.0)
    else:
        k = oracle.BC_CHARACTERISTIC if kind == "characteristic" else oracle.BC_OUTFLOW
        bc, v = [k] * 4, (speed * 0.8, -speed * 0.6)
    x0 = states.conservative(*[np.array([q]) for q in (0.9, v[0], v[1], 1.1)], G)[0]
    M = oracle.Mesh(3, *spec.args(), bc=bc, ext=np.tile(x0, (4, 1)))
    x, y, m = M.geometry()
    u0 = states.constant(x, rho=0.9, v1=v[0], v2=v[1], p=1.1)
    u = u0
    for _ in range(3):
        u, st = M.ssprk3(u, 0.9, limiter=oracle.LIM_LOCAL)
    assert state_err(u, u0) < 1e-13


def test_ghost_rules(oracle):
    """The ghost states follow their stated rules (an interface check of the
    branches, not a pin): wall reverses the normal momentum only; the
    characteristic branches by the outward normal Mach number."""
    rng = np.random.default_rng(3)
    for _ in range(200):
        f = int(rng.integers(4))
        r, p = rng.uniform(0.2, 2), rng.uniform(0.2, 2)
        c = np.sqrt(G * p / r)
        vn = rng.uniform(-2, 2) * c
        vt = rng.uniform(-1, 1)
        sgn = 1.0 if f & 1 else -1.0
        vel = [0.0, 0.0]
        vel[f // 2], vel[1 - f // 2] = sgn * vn, vt
        ui = states.conservative(*[np.array([q]) for q in (r, vel[0], vel[1], p)], G)[0]
        re, pe = rng.uniform(0.2, 2), rng.uniform(0.2, 2)
        ve = rng.uniform(-1, 1, 2)
        ue = states.conservative(*[np.array([q]) for q in (re, ve[0], ve[1], pe)], G)[0]
        gw = oracle.boundary_ghost(oracle.BC_WALL, ue, ui, f)
        want = ui.copy()
        want[1 + f // 2] *= -1
        assert np.array_equal(gw, want)
        assert np.array_equal(oracle.boundary_ghost(oracle.BC_OUTFLOW, ue, ui, f), ui)
        g = oracle.boundary_ghost(oracle.BC_CHARACTERISTIC, ue, ui, f)
        gr, gv1, gv2 = g[0], g[1] / g[0], g[2] / g[0]
        gp = (G - 1) * (g[3] - 0.5 * gr * (gv1 ** 2 + gv2 ** 2))
        if vn <= -c:
            assert np.allclose(g, ue, rtol=1e-14, atol=0)
        elif vn <= 0:
            assert np.allclose([gr, gv1, gv2, gp], [re, ve[0], ve[1], p], rtol=1e-12, atol=1e-14)
        elif vn < c:
            assert np.allclose([gr, gv1, gv2, gp], [r, vel[0], vel[1], pe], rtol=1e-12, atol=1e-14)
        else:
            assert np.array_equal(g, ui)


def test_boundary_node_numbering(oracle):
    """Boundary nodes are numbered by (element, face, node along the face), one
    block of N+1 per boundary face; opposite sides must agree on periodicity."""
    spec = random_mesh(2, 4, 2, 0.4)
    M = oracle.Mesh(3, *spec.args(), bc=[2, 3, 0, 0])
    bn = M.boundary_nodes()
    key = bn[:, 0] * 16 + bn[:, 1] * 4 + bn[:, 2]
    assert np.all(np.diff(key) > 0) and set(bn[:, 1]) == {0, 1}
    x, y, _ = M.geometry()
    xs = np.array([x[e, 0, 0] if f == 0 else x[e, 0, -1] for e, f, k in bn])
    assert np.allclose(xs[bn[:, 1] == 0], 0.0) and np.allclose(xs[bn[:, 1] == 1], 1.0)
    assert M.faces()[:, :, 0].max() == 3
    with pytest.raises(ValueError):
        oracle.Mesh(3, *spec.args(), bc=[1, 0, 0, 0])
    with pytest.raises(ValueError):
        M.set_boundary_states(np.zeros(M.NB, np.int8), np.zeros((M.NB, 4)))
