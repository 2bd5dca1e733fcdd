"""GPU non-periodic boundaries (slip wall, characteristic inflow/outflow, outflow;
the conditions of Sec. 3.5 and 3.6) against the oracle, through the C-ABI.

Tolerances: 1e-12 per DOF (the state metric of parity.py) for residuals and for
single limited forward-Euler steps; whole runs with local limiting are compared
in relative L1 (< 1e-9), since local factors are discontinuous where a node sits
on its bound."""
import numpy as np
import pytest

from parity import rate_err, state_err
from workloads import states
from workloads.meshes import random_mesh

pytestmark = pytest.mark.gpu
TOL = 1e-12
G = 1.4


def _cons(r, v1, v2, p):
    return states.conservative(*[np.array([q], dtype=float) for q in (r, v1, v2, p)], G)[0]


def pair(oracle, spec, N, bc, ext=None, limiter=None, **kw):
    import paper_2607_06045_amd as P
    s = P.Solver(N, limiter=P.LIMIT_POSITIVITY if limiter is None else limiter, bc=bc, ext=ext, **kw)
    s.set_mesh(*spec.args())
    M = oracle.Mesh(N, *spec.args(), bc=bc, ext=ext)
    assert (s.E, s.M, s.NB) == (M.E, M.M, M.NB)
    assert np.array_equal(s.boundary_nodes(), M.boundary_nodes())
    # the host-only check agrees with the uploaded mesh
    assert P.validate_mesh_bc(N, spec.level, spec.ix, spec.iy, spec.nx0, spec.ny0, bc=bc) == (s.M, s.NB)
    return s, M


def _mixed_states(M, seed):
    """Per-node conditions and exterior states: every kind, and exterior flows
    that make the characteristic nodes take all four branches."""
    rng = np.random.default_rng(seed)
    kind = rng.integers(1, 4, M.NB).astype(np.int8)
    ext = np.stack([_cons(rng.uniform(0.5, 1.5), rng.uniform(-2.5, 2.5), rng.uniform(-2.5, 2.5),
                          rng.uniform(0.5, 1.5)) for _ in range(M.NB)])
    return kind, ext


def _flow(x, y, seed):
    rng = np.random.default_rng(seed)
    k = rng.uniform(1, 3, 4)
    rho = 1.0 + 0.3 * np.sin(k[0] * x + 0.4) * np.cos(k[1] * y)
    v1 = 1.6 * np.sin(k[2] * y + 0.3)  # sub- and supersonic normal speeds at the sides
    v2 = -1.4 * np.cos(k[3] * x)
    p = 1.0 + 0.2 * np.cos(k[0] * x * y)
    return states.conservative(rho, v1, v2, p, G)


CASES = ["walls", "characteristic", "mixed-nodes", "x-walls-y-periodic"]


def _setup(oracle, name, N, limiter=None):
    spec = random_mesh(10, 6, 2, 0.4, L=2.0, x0=-1.0, y0=-1.0)
    ext = np.tile(_cons(1.1, 0.8, -0.3, 0.9), (4, 1))
    ext[0] = _cons(1.3, 2.2, 0.1, 1.0)  # supersonic inflow on x-
    if name == "walls":
        bc = [1, 1, 1, 1]
    elif name == "x-walls-y-periodic":
        bc = [1, 1, 0, 0]
    else:
        bc = [2, 3, 2, 2]
    s, M = pair(oracle, spec, N, bc, ext, limiter)
    if name == "mixed-nodes":
        kind, bext = _mixed_states(M, 4)
        s.set_boundary_states(kind, bext)
        M.set_boundary_states(kind, bext)
    return s, M


@pytest.mark.parametrize("N", [3, 4])
@pytest.mark.parametrize("name", CASES)
def test_boundary_rhs_and_dt_parity(oracle, name, N):
    s, M = _setup(oracle, name, N)
    x, y, m = M.geometry()
    u = _flow(x, y, 1)
    s.upload(u)
    w0 = oracle.basis(N)[1][0]
    for which in (oracle.RHS_HIGH, oracle.RHS_LOW):
        err = rate_err(s.rhs(which), M.rhs(u, which), u, x, y, w0)
        print(f"boundary {name} N={N} rhs {which} err={err:.2e}", flush=True)
        assert err < TOL
    dg, dc = s.max_dt(0.9), M.max_dt(u, 0.9)
    assert abs(dg - dc) <= 1e-13 * dc


@pytest.mark.parametrize("N", [3, 4])
@pytest.mark.parametrize("limiter", ["positivity", "local", "combined"])
@pytest.mark.parametrize("name", CASES)
def test_boundary_limited_step_parity(oracle, name, limiter, N):
    import paper_2607_06045_amd as P
    lim = {"positivity": P.LIMIT_POSITIVITY, "local": P.LIMIT_LOCAL, "combined": P.LIMIT_COMBINED}[limiter]
    s, M = _setup(oracle, name, N, lim)
    x, y, m = M.geometry()
    u = _flow(x, y, 2)
    s.upload(u)
    dt = M.max_dt(u, 0.9)
    st = s.limit(dt)
    c, sc = M.fe_step(u, dt, limiter=lim)
    err = state_err(s.download(), c)
    print(f"boundary {name} {limiter} N={N} fe err={err:.2e} theta={sc['theta_vol_min']:.3f}", flush=True)
    assert err < TOL
    assert st["violations"] == 0 and sc["violations"] == 0


@pytest.mark.parametrize("limiter", ["positivity", "local"])
def test_closed_box_blast_run(oracle, limiter):
    """A blast that hits the walls of a closed box, four SSP-RK3 steps of the GPU
    on its own: mass and energy conserved, no bound violations, the state close
    to the oracle's run."""
    import paper_2607_06045_amd as P
    lim = P.LIMIT_POSITIVITY if limiter == "positivity" else P.LIMIT_LOCAL
    spec = random_mesh(4, 6, 2, 0.4, L=1.0, x0=-0.5, y0=-0.5)
    s, M = pair(oracle, spec, 3, [1, 1, 1, 1], limiter=lim)
    x, y, m = M.geometry()
    u = states.sedov_tophat(x - 0.1, y + 0.3, r0=0.15)
    s.upload(u)
    c = u
    tot0 = (u * m[:, None]).sum(axis=(0, 2, 3))
    for _ in range(4):
        st = s.step(0.5)
        c, sc = M.ssprk3(c, 0.5, limiter=lim)
        assert st["violations"] == 0 and sc["violations"] == 0
    g = s.download()
    scale = (np.abs(g) * m[:, None]).sum(axis=(0, 2, 3))
    cons = np.abs((g * m[:, None]).sum(axis=(0, 2, 3)) - tot0) / scale
    l1 = (np.abs(g - c) * m[:, None]).sum(axis=(0, 2, 3)) / scale
    print(f"closed box {limiter}: max err {state_err(g, c):.2e} rel L1 {l1} conservation {cons}",
          flush=True)
    assert cons[0] < 1e-13 and cons[3] < 1e-13
    if limiter == "positivity":
        assert state_err(g, c) < TOL
    assert l1.max() < 1e-9


def test_boundary_arguments():
    """Errors of the boundary entry points: mixed periodicity, an unknown
    condition, an inadmissible exterior state, boundaries after the mesh, bad
    per-node conditions (which leave the states unchanged)."""
    import paper_2607_06045_amd as P
    good = np.tile(_cons(1.0, 0.5, 0.0, 1.0), (4, 1))
    for bc, ext in (([1, 0, 0, 0], None), ([4, 4, 0, 0], None), ([2, 2, 0, 0], None),
                    ([2, 2, 0, 0], np.tile(_cons(1.0, 0.5, 0.0, -1.0), (4, 1)))):
        with pytest.raises(P.DgidpError):
            P.Solver(3, bc=bc, ext=ext)
    spec = random_mesh(1, 4, 1, 0.3)
    s = P.Solver(3, bc=[2, 2, 1, 1], ext=good)
    s.set_mesh(*spec.args())
    assert s.NB > 0
    with pytest.raises(P.DgidpError):
        s.set_boundary_states(np.zeros(s.NB, np.int8), np.tile(good[0], (s.NB, 1)))
    bad = np.tile(good[0], (s.NB, 1))
    bad[3, 0] = -1.0
    with pytest.raises(P.DgidpError):
        s.set_boundary_states(np.full(s.NB, 2, np.int8), bad)
    s.set_boundary_states(np.full(s.NB, 1, np.int8), bad)  # walls ignore the exterior state
    from paper_2607_06045_amd import _lib
    b = np.array([0, 0, 0, 0], np.int32)
    assert _lib._lib.dgidp_set_boundaries(s._h, b.ctypes.data, None) == -1


def test_double_mach_reflection_short():
    """The double Mach reflection (Sec. 3.5) at 64 x 20 elements, N = 4, to
    t = 0.05: the incident shock is straight and moves at a known speed, so its
    position on the upper side (characteristic boundary against the exact moving
    shock) is exact: within two cell widths.  No bound violations; the density
    stays above the pre-shock value up to the limiter's tolerance."""
    from paper_2607_06045_amd.evaluate import run_dmr
    r = run_dmr(level=2, t_end=0.05)
    print(r, flush=True)
    assert r["violations"] == 0
    assert r["rho_min"] > 1.4 * (1 - 1e-3) and r["p_min"] > 0.99
    assert len(r["top_shock_x"]) == 1
    assert abs(r["top_shock_x"][0] - r["top_shock_x_exact"]) < 2 * r["hx"]


def test_jet_short():
    """The Mach-2000 jet (Sec. 3.6: gamma = 5/3, Chandrashekar flux, combined
    limiting, characteristic inflow band) at 32 x 32 elements to t = 5e-4: no
    bound violations, no inadmissible low-order state, positive density and
    pressure, and the jet has entered the domain."""
    from paper_2607_06045_amd.evaluate import run_jet
    r = run_jet(level=5, t_end=5e-4)
    print(r, flush=True)
    assert r["violations"] == 0 and r["fv_inadmissible"] == 0
    assert r["rho_min"] > 0 and r["p_min"] > 0
    assert r["jet_head_x"] is not None and r["jet_head_x"] > -0.3
