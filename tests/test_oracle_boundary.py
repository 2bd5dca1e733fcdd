"""Pins of the oracle's non-periodic boundaries: slip walls and characteristic
inflow/outflow, the conditions of the double Mach reflection and the jet
(Sec. 3.5, 3.6).

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
- The subsonic characteristic branches against characteristic theory:
  a uniform-velocity, uniform-pressure flow stays so to rounding under every
  flux, mortar and limiter of the scheme (momentum and energy are linear in the
  density at fixed velocity and pressure), so a contact entering through a
  subsonic inflow and one leaving through a subsonic outflow keep velocity and
  pressure exact whatever the ignored exterior values are; at the matching
  pressure the subsonic outflow is the plain outflow; a subsonic inflow that
  imposes a lower speed sends in a rarefaction that keeps the outgoing
  invariant u - 2c/(gamma-1); a subsonic outflow that imposes a lower pressure
  sends in one that keeps u + 2c/(gamma-1) and the entropy."""
import numpy as np
import pytest

from parity import state_err
from workloads import states
from workloads.meshes import MeshSpec, random_mesh, refined_box_mesh, uniform_mesh

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


def _channel_run(oracle, axis, sign, ext_lo, ext_hi, rho0, T, limiter=None, bc_hi=None):
    """A channel of 64 x 4 square elements (N=3) along the axis, periodic across
    it, characteristic on both ends (bc_hi overrides the upper end); the flow
    runs along the axis at speed sign * 0.5 with pressure 1 and density rho0(s)
    (s the coordinate along the axis).  ext_lo / ext_hi are the exterior
    states of the two ends as (rho, velocity along, velocity across, p).
    Returns s and the primitive variables (rho, along, across, p) at T."""
    lim = oracle.LIM_POSITIVITY if limiter is None else limiter
    spec = uniform_mesh(64, 4, Lx=1.0, Ly=1 / 16) if axis == 0 else uniform_mesh(4, 64, Lx=1 / 16, Ly=1.0)

    def cons(r, un, ut, p):
        v = (un, ut) if axis == 0 else (ut, un)
        return states.conservative(*[np.array([q]) for q in (r, v[0], v[1], p)], G)[0]

    lo, hi = (0, 1) if axis == 0 else (2, 3)
    ext = np.zeros((4, 4))
    ext[lo], ext[hi] = cons(*ext_lo), cons(*ext_hi)
    bc = [0, 0, 0, 0]
    bc[lo] = oracle.BC_CHARACTERISTIC
    bc[hi] = oracle.BC_CHARACTERISTIC if bc_hi is None else bc_hi
    M = oracle.Mesh(3, *spec.args(), bc=bc, ext=ext)
    x, y, _ = M.geometry()
    s = x if axis == 0 else y
    un, ut = sign * 0.5 + 0 * s, 0 * s
    v = (un, ut) if axis == 0 else (ut, un)
    u = states.conservative(rho0(s), v[0], v[1], 1.0 + 0 * s, G)
    t = 0.0
    while t < T * (1 - 1e-12):
        dt = min(M.max_dt(u, 0.5), T - t)
        u, st = M.ssprk3_dt(u, dt, limiter=lim)
        assert st["violations"] == 0 and st["fv_inadmissible"] == 0
        t += dt
    r = u[:, 0]
    v1, v2 = u[:, 1] / r, u[:, 2] / r
    p = (G - 1) * (u[:, 3] - 0.5 * r * (v1 ** 2 + v2 ** 2))
    return (s, r, v1, v2, p) if axis == 0 else (s, r, v2, v1, p)


@pytest.mark.parametrize("limiter", ["positivity", "local"])
@pytest.mark.parametrize("axis,sign", [(0, 1), (0, -1), (1, 1), (1, -1)])
def test_subsonic_contact_passes_both_ends(oracle, axis, sign, limiter):
    """Density 2 enters through the subsonic inflow, whose exterior pressure (3)
    must be ignored; a density bump leaves through the subsonic outflow, whose
    exterior density and velocity (5; -0.3 and 0.7) must be ignored.  Velocity
    and pressure stay exact; the density at the inflow end approaches 2."""
    lim = oracle.LIM_POSITIVITY if limiter == "positivity" else oracle.LIM_LOCAL
    inflow = (2.0, sign * 0.5, 0.0, 3.0)
    outflow = (5.0, -0.3 * sign, 0.7, 1.0)
    s_out = 0.95 if sign > 0 else 0.05
    s, r, un, ut, p = _channel_run(oracle, axis, sign, *((inflow, outflow) if sign > 0 else (outflow, inflow)),
                                   lambda s: 1.0 + 0.3 * np.exp(-((s - s_out) / 0.05) ** 2), 0.05, lim)
    errs = np.abs(un - sign * 0.5).max(), np.abs(ut).max(), np.abs(p - 1.0).max()
    near_in = s < 0.015 if sign > 0 else s > 0.985
    print(f"contact axis {axis} sign {sign} {limiter}: |un - U| {errs[0]:.1e}, |ut| {errs[1]:.1e}, "
          f"|p - 1| {errs[2]:.1e}; density at the inflow {r[near_in].mean():.4f}")
    assert max(errs) < 1e-13
    assert r[near_in].mean() > 1.9


@pytest.mark.parametrize("axis", [0, 1])
def test_subsonic_outflow_at_matching_pressure_is_plain_outflow(oracle, axis):
    """At the interior pressure the subsonic outflow's ghost is the interior
    state (up to the rounding of its energy), so the run equals the run with a
    plain outflow there."""
    inflow, outflow = (2.0, 0.5, 0.0, 3.0), (5.0, -0.3, 0.7, 1.0)
    bump = lambda s: 1.0 + 0.3 * np.exp(-((s - 0.95) / 0.05) ** 2)
    a = _channel_run(oracle, axis, 1, inflow, outflow, bump, 0.03)
    b = _channel_run(oracle, axis, 1, inflow, outflow, bump, 0.03, bc_hi=oracle.BC_OUTFLOW)
    err = max(np.abs(qa - qb).max() for qa, qb in zip(a[1:], b[1:]))
    print(f"axis {axis}: characteristic outflow vs plain outflow {err:.1e}")
    assert err < 1e-12


@pytest.mark.parametrize("axis", [0, 1])
def test_subsonic_inflow_rarefaction(oracle, axis):
    """The inflow end imposes density 1 and speed 0.45 (exterior pressure 7,
    ignored) on the flow (1, 0.5, p = 1).  A rarefaction runs in; the outgoing
    characteristics keep u - 2c/(gamma-1), so behind it, next to the end,
    u = 0.45, rho = 1 and c = c0 + (gamma-1)/2 (0.45 - 0.5), p = (c/c0)^(2 gamma/(gamma-1))."""
    Ue = 0.45
    s, r, un, ut, p = _channel_run(oracle, axis, 1, (1.0, Ue, 0.0, 7.0), (1.0, 0.5, 0.0, 1.0),
                                   lambda s: 1.0 + 0 * s, 0.2)
    c0 = np.sqrt(G)
    cm = c0 + 0.5 * (G - 1) * (Ue - 0.5)
    pm = (cm / c0) ** (2 * G / (G - 1))
    reg = s < 0.03  # the contact is at 0.09
    e = np.abs(un[reg] - Ue).max(), np.abs(p[reg] - pm).max(), np.abs(r[reg] - 1.0).max()
    print(f"inflow rarefaction axis {axis}: u {e[0]:.1e}, p {e[1]:.1e} (jump {1 - pm:.3f}), rho {e[2]:.1e}")
    # the wave changes u by 0.05 and p by 0.058; the discretisation error at
    # this resolution is about 1e-4
    assert max(e) < 1e-3


@pytest.mark.parametrize("axis", [0, 1])
def test_subsonic_outflow_rarefaction(oracle, axis):
    """The outflow end imposes pressure 0.95 (exterior density 3 and velocity
    (-1, 0.4) ignored) on the flow (1, 0.5, p = 1).  A rarefaction runs in; the
    outgoing characteristics keep u + 2c/(gamma-1) and the entropy, so next to
    the end p = 0.95, rho = 0.95^(1/gamma) and u = 0.5 + 2 (c0 - c)/(gamma-1)."""
    pe = 0.95
    s, r, un, ut, p = _channel_run(oracle, axis, 1, (1.0, 0.5, 0.0, 1.0), (3.0, -1.0, 0.4, pe),
                                   lambda s: 1.0 + 0 * s, 0.2)
    rb = pe ** (1 / G)
    cb = np.sqrt(G * pe / rb)
    ub = 0.5 + 2 * (np.sqrt(G) - cb) / (G - 1)
    reg = s > 0.95  # the rarefaction's tail is at 0.87
    e = np.abs(un[reg] - ub).max(), np.abs(p[reg] - pe).max(), np.abs(r[reg] - rb).max(), np.abs(ut).max()
    print(f"outflow rarefaction axis {axis}: u {e[0]:.1e} (jump {ub - 0.5:.3f}), p {e[1]:.1e}, rho {e[2]:.1e}, "
          f"|ut| {e[3]:.1e}")
    assert max(e[:3]) < 1e-3 and e[3] < 1e-13


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
