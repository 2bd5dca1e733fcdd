"""GPU mesh adaptation (Sec. 2.4) against the oracle, through the C-ABI:
the adapted leaf list (bit-exact), the transferred state (interpolation and
L2 projection, 1e-12 per the state metric), the Zhang-Shu transfer limiter,
and SSP-RK3 steps on the adapted mesh."""
import numpy as np
import pytest

from parity import state_err
from workloads import states
from workloads.meshes import workload_mesh, random_flags, random_mesh, to_spec

pytestmark = pytest.mark.gpu
TOL = 1e-12


def _setup(oracle, spec, N, u_fn):
    import paper_2607_06045_amd as P
    s = P.Solver(N)
    s.set_mesh(*spec.args())
    M = oracle.Mesh(N, *spec.args())
    x, y, m = M.geometry()
    u = u_fn(x, y)
    s.upload(u)
    return s, M, u


@pytest.mark.parametrize("N", [3, 4])
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_transfer_parity(oracle, N, seed):
    spec = random_mesh(seed, 4, 3, 0.4)
    s, M, u = _setup(oracle, spec, N, lambda x, y: states.density_wave(x, y))
    flags = random_flags(spec, 20 + seed, p_refine=0.15, p_coarsen=0.6)
    st = s.refine_coarsen(flags, zs_eps=1e-10)
    nl, nx, ny, kind, src = oracle.adapt(spec.level, spec.ix, spec.iy, spec.nx0, spec.ny0, flags)
    lv, ix, iy = s.mesh()
    assert np.array_equal(lv, nl) and np.array_equal(ix, nx) and np.array_equal(iy, ny)
    ref, nlim, nbad = oracle.transfer(N, kind, src, u, eps=1e-10)
    err = state_err(s.download(), ref)
    print(f"transfer N={N} seed={seed}: {spec.E} -> {len(nl)} leaves {st}, err={err:.2e}", flush=True)
    assert st["zs_limited"] == nlim == 0
    assert (kind == 1).any() and (kind == 2).any()
    assert err < TOL
    # mass is kept
    m1 = oracle.Mesh(N, nl, nx, ny, *spec.args()[3:]).geometry()[2]
    m0 = M.geometry()[2]
    t0 = (m0[:, None] * u).sum(axis=(0, 2, 3))
    t1 = (m1[:, None] * s.download()).sum(axis=(0, 2, 3))
    assert np.abs(t1 - t0).max() < 1e-13 * np.abs(t0).max()


@pytest.mark.parametrize("N", [3, 4])
def test_zhang_shu_parity(oracle, N):
    """A sharp near-vacuum blast inside one element of a uniform mesh: its
    children undershoot, the limiter scales them back toward the parent mean."""
    spec = to_spec((0.0, 0.0, 1.0, 1.0, 4, 4), {(0, i, j) for i in range(4) for j in range(4)})

    def u_fn(x, y):
        r2 = (x - 0.58) ** 2 + (y - 0.6) ** 2
        rho = 5e-3 + np.exp(-r2 / 0.002)
        p = 5e-3 + 5.0 * np.exp(-((x - 0.4) ** 2 + (y - 0.45) ** 2) / 0.001)
        return states.conservative(rho, 0.4 + 0 * x, -0.2 + 0 * x, p, 1.4)

    s, M, u = _setup(oracle, spec, N, u_fn)
    flags = np.zeros(spec.E, np.int8)
    flags[:] = 1
    eps = 1e-3
    st = s.refine_coarsen(flags, zs_eps=eps)
    nl, nx, ny, kind, src = oracle.adapt(spec.level, spec.ix, spec.iy, 4, 4, flags)
    ref, nlim, nbad = oracle.transfer(N, kind, src, u, eps=eps)
    g = s.download()
    err = state_err(g, ref)
    p = 0.4 * (g[:, 3] - 0.5 * (g[:, 1] ** 2 + g[:, 2] ** 2) / g[:, 0])
    print(f"zhang-shu N={N}: {st}, oracle limited {nlim}, err={err:.2e}, min rho {g[:, 0].min():.3e} "
          f"min p {p.min():.3e}", flush=True)
    assert nlim > 0 and st["zs_limited"] == nlim and st["zs_unfixable"] == nbad == 0
    assert (g[:, 0] >= eps).all() and (p >= eps).all()
    assert err < TOL


def test_step_after_adaptation(oracle):
    """The adapted mesh has new mortars; stepping on it matches the oracle."""
    import paper_2607_06045_amd as P
    spec = workload_mesh("vortex304")
    s, M, u = _setup(oracle, spec, 3, lambda x, y: states.workload_state("vortex304", x, y))
    flags = random_flags(spec, 4, p_refine=0.1, p_coarsen=0.7)
    s.refine_coarsen(flags)
    lv, ix, iy = s.mesh()
    M2 = oracle.Mesh(3, lv, ix, iy, *spec.args()[3:])
    u2 = s.download()
    assert (s.E, s.M) == (M2.E, M2.M)
    st = s.step(0.5)
    ref, _ = M2.ssprk3(u2, 0.5)
    err = state_err(s.download(), ref)
    print(f"step after adaptation: {spec.E} -> {s.E} leaves, {s.M} mortars, err={err:.2e}", flush=True)
    assert st["violations"] == 0 and err < TOL


def test_refine_then_coarsen_back(oracle):
    """Refining every leaf and then coarsening the new sibling groups returns
    the mesh, its leaf order and, up to round-off, the state (projection of
    the interpolant).  Coarsening is checked against the levels before the
    pass, so groups next to finer groups wait for a later pass."""
    import paper_2607_06045_amd as P
    spec = random_mesh(7, 4, 2, 0.3)
    s, M, u = _setup(oracle, spec, 3, lambda x, y: states.vortex(x, y))
    s.refine_coarsen(np.ones(spec.E, np.int8))
    orig = set(zip(spec.level.tolist(), spec.ix.tolist(), spec.iy.tolist()))
    passes = 0
    while s.E != spec.E:
        lv, ix, iy = s.mesh()
        flags = np.array([-1 if (l - 1, i >> 1, j >> 1) in orig else 0
                          for l, i, j in zip(lv.tolist(), ix.tolist(), iy.tolist())], np.int8)
        before = s.E
        s.refine_coarsen(flags)
        passes += 1
        assert s.E < before and passes <= 4
    lv, ix, iy = s.mesh()
    assert np.array_equal(lv, spec.level) and np.array_equal(ix, spec.ix) and np.array_equal(iy, spec.iy)
    err = state_err(s.download(), u)
    print(f"refine + {passes} coarsening passes: state err {err:.2e}", flush=True)
    assert err < TOL


def test_refine_coarsen_errors():
    import paper_2607_06045_amd as P
    spec = random_mesh(1, 4, 1, 0.3)
    s = P.Solver(3)
    s.set_mesh(*spec.args())
    with pytest.raises(P.DgidpError):
        s.refine_coarsen(np.zeros(spec.E, np.int8))  # no state yet
    x, y = s.node_coords()
    s.upload(states.vortex(x, y))
    with pytest.raises(ValueError):
        s.refine_coarsen(np.zeros(spec.E + 1, np.int8))
    with pytest.raises(P.DgidpError):
        s.refine_coarsen(np.zeros(spec.E, np.int8), zs_eps=-1.0)


@pytest.mark.parametrize("N", [3, 4])
def test_adaptation_with_walls(oracle, N):
    """Adaptation on a mesh with slip walls and characteristic sides: the same
    leaf list and transferred state as the oracle (the balance rules are those
    of the periodic domain), the boundary nodes of the new mesh numbered as the
    oracle numbers them and reset to the side settings, and a step on the
    adapted mesh equal to the oracle's."""
    import paper_2607_06045_amd as P
    spec = random_mesh(2, 4, 3, 0.4)
    ext = np.tile(np.array([1.0, 0.3, -0.1, 2.5]), (4, 1))
    bc = [P.BC_WALL, P.BC_WALL, P.BC_CHARACTERISTIC, P.BC_OUTFLOW]
    s = P.Solver(N, bc=bc, ext=ext)
    s.set_mesh(*spec.args())
    M = oracle.Mesh(N, *spec.args(), bc=bc, ext=ext)
    x, y, m = M.geometry()
    u = states.density_wave(x, y)
    s.upload(u)
    s.set_boundary_states(np.full(s.NB, P.BC_WALL, np.int8), np.tile(ext[0], (s.NB, 1)))
    flags = random_flags(spec, 31, p_refine=0.2, p_coarsen=0.6)
    s.refine_coarsen(flags, zs_eps=1e-10)
    nl, nx, ny, kind, src = oracle.adapt(spec.level, spec.ix, spec.iy, spec.nx0, spec.ny0, flags)
    lv, ix, iy = s.mesh()
    assert np.array_equal(lv, nl) and np.array_equal(ix, nx) and np.array_equal(iy, ny)
    ref, _, _ = oracle.transfer(N, kind, src, u, eps=1e-10)
    assert state_err(s.download(), ref) < TOL
    M2 = oracle.Mesh(N, nl, nx, ny, *spec.args()[3:], bc=bc, ext=ext)
    assert (s.E, s.M, s.NB) == (M2.E, M2.M, M2.NB)
    assert np.array_equal(s.boundary_nodes(), M2.boundary_nodes())
    u2 = s.download()
    dt = M2.max_dt(u2, 0.5)
    st = s.step_dt(dt)
    c, sc = M2.ssprk3_dt(u2, dt)
    err = state_err(s.download(), c)
    print(f"adaptation with walls N={N}: {spec.E} -> {s.E} leaves, NB {s.NB}, step err={err:.2e}", flush=True)
    assert err < TOL and st["violations"] == 0


@pytest.mark.parametrize("N", [3, 4])
def test_zhang_shu_jet_edges(oracle, N):
    """Refinement of elements that hold the edge of a hypersonic jet (gamma =
    5/3, pressure a 1e-7 part of the energy): every pressure stays at or above
    the threshold 1e-10, and the limited transfer equals the oracle's within
    1e-10.  The scaling factor solves a pressure quadratic whose coefficients
    cancel from the energy scale (1e6) down to the pressure (1e-1), so its
    rounding is amplified by up to E/p ~ 1e7 over the unit roundoff, about
    1e-9 in theta at worst (measured: 1.4e-12 in the state metric)."""
    import paper_2607_06045_amd as P
    g = 5.0 / 3.0
    spec = to_spec((0.0, 0.0, 1.0, 1.0, 4, 4), {(0, i, j) for i in range(4) for j in range(4)})
    M = oracle.Mesh(N, *spec.args())
    x, y, m = M.geometry()
    rng = np.random.default_rng(11)
    u = np.empty((spec.E, 4, N + 1, N + 1))
    for e in range(spec.E):
        xi = 2 * (x[e] - x[e].min()) / (x[e].max() - x[e].min()) - 1
        eta = 2 * (y[e] - y[e].min()) / (y[e].max() - y[e].min()) - 1
        y0, d, ang = rng.uniform(-0.6, 0.6), rng.uniform(0.01, 0.1), rng.uniform(0, np.pi)
        sgm = 0.5 * (1 + np.tanh((np.cos(ang) * eta + np.sin(ang) * xi - y0) / d))
        rj, v, p = rng.uniform(2, 10), rng.uniform(200, 1000), rng.uniform(0.1, 1.0)
        u[e] = states.conservative((0.5 + (rj - 0.5) * sgm)[None], (v * sgm)[None], 0 * sgm[None],
                                   p + 0 * sgm[None], g)[0]
    s = P.Solver(N, gamma=g)
    s.set_mesh(*spec.args())
    s.upload(u)
    flags = np.ones(spec.E, np.int8)
    st = s.refine_coarsen(flags, zs_eps=1e-10)
    nl, nx, ny, kind, src = oracle.adapt(spec.level, spec.ix, spec.iy, 4, 4, flags)
    ref, nlim, nbad = oracle.transfer(N, kind, src, u, eps=1e-10, gamma=g)
    gpu = s.download()
    pg = (g - 1) * (gpu[:, 3] - 0.5 * (gpu[:, 1] ** 2 + gpu[:, 2] ** 2) / gpu[:, 0])
    err = state_err(gpu, ref)
    print(f"jet-edge transfer N={N}: {st}, oracle limited {nlim}, err={err:.2e}, min p {pg.min():.3e}", flush=True)
    assert nlim == spec.E and st["zs_limited"] == nlim and st["zs_unfixable"] == nbad == 0
    assert (gpu[:, 0] >= 1e-10).all() and (pg >= 1e-10).all()
    assert err < 1e-10
