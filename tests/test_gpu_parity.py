"""GPU (HIP, gfx950) against the oracle, through the C-ABI, FP64 path.

Tolerance: 1e-12 relative per DOF (states) and per variable scale (rates)."""
import numpy as np
import pytest

from parity import rate_err, state_err
from workloads import states
from workloads.meshes import workload_mesh, random_mesh, refined_box_mesh

pytestmark = pytest.mark.gpu
TOL = 1e-12


def pair(oracle, spec, N=3, gamma=1.4, **kw):
    import paper_2607_06045_amd as P
    s = P.Solver(N, gamma=gamma, **kw)
    s.set_mesh(*spec.args())
    M = oracle.Mesh(N, *spec.args())
    assert (s.E, s.M) == (M.E, M.M)
    return s, M


MESHES = {
    "vortex304": lambda: workload_mesh("vortex304"),
    "random0": lambda: random_mesh(0, 4, 3, 0.4),
    "random3": lambda: random_mesh(3, 4, 3, 0.4),
}


def smooth_state(kind, x, y):
    if kind == "vortex":
        return states.vortex(x, y)
    return states.density_wave(x, y)


@pytest.mark.parametrize("N", [3, 4])
@pytest.mark.parametrize("name", sorted(MESHES))
def test_rhs_parity(oracle, name, N):
    s, M = pair(oracle, MESHES[name](), N)
    x, y, m = M.geometry()
    xg, yg = s.node_coords()
    assert np.abs(xg - x).max() < 1e-14 and np.abs(yg - y).max() < 1e-14
    u = states.vortex(x, y) if name == "vortex304" else states.density_wave(x, y)
    s.upload(u)
    assert np.array_equal(s.download(), u)
    w0 = oracle.basis(N)[1][0]
    for which in (0, 1):
        g = s.rhs(which)
        c = M.rhs(u, which)
        err = rate_err(g, c, u, x, y, w0)
        print(f"rhs {name} N={N} which={which} err={err:.2e}", flush=True)
        assert err < TOL


@pytest.mark.parametrize("N", [3, 4])
def test_dt_parity(oracle, N):
    import paper_2607_06045_amd as P
    spec = random_mesh(1, 4, 3, 0.4)
    for mode in (P.DT_IDP, P.DT_LOWORDER):
        s, M = pair(oracle, spec, N, dt_mode=mode)
        x, y, m = M.geometry()
        u = states.random_admissible(x, 3, rho_range=(0.5, 1.5), p_range=(0.5, 1.5), vmax=0.5)
        s.upload(u)
        g, c = s.max_dt(0.7), M.max_dt(u, 0.7, mode)
        print(f"dt N={N} mode={mode} gpu={g!r} oracle={c!r}", flush=True)
        assert abs(g - c) <= 1e-14 * c


@pytest.mark.parametrize("N", [3, 4])
@pytest.mark.parametrize("name", ["vortex304", "random3"])
def test_limited_forward_euler_parity(oracle, name, N):
    s, M = pair(oracle, MESHES[name](), N)
    x, y, m = M.geometry()
    u = states.vortex(x, y) if name == "vortex304" else states.density_wave(x, y)
    s.upload(u)
    dt = M.max_dt(u, 0.9)
    st = s.limit(dt)
    c, sc = M.fe_step(u, dt)
    err = state_err(s.download(), c)
    print(f"fe {name} N={N} err={err:.2e} stats={st}", flush=True)
    assert err < TOL
    assert st["violations"] == 0 and sc["violations"] == 0


@pytest.mark.parametrize("N", [3, 4])
def test_blast_steps_parity(oracle, N):
    """Top-hat blast: the limiter acts in the volume and at the mortars, and some
    mortars fall back to the low-order flux (inadmissible interpolated states)."""
    spec = random_mesh(10, 8, 2, 0.45, L=4.0, x0=-2.0, y0=-2.0)
    s, M = pair(oracle, spec, N)
    x, y, m = M.geometry()
    u = states.sedov_tophat(x, y, r0=0.5)
    s.upload(u)
    c = u
    for k in range(3):
        st = s.step(0.9)
        c, sc = M.ssprk3(c, 0.9)
        assert abs(st["dt"] - sc["dt"]) <= 1e-13 * sc["dt"]
        err = state_err(s.download(), c)
        print(f"blast N={N} step {k} err={err:.2e} gpu={st} oracle={sc}", flush=True)
        assert err < TOL
        assert st["violations"] == 0
        assert abs(st["theta_vol_min"] - sc["theta_vol_min"]) < 1e-10
        assert abs(st["theta_mort_min"] - sc["theta_mort_min"]) < 1e-10
    assert sc["theta_vol_min"] < 0.5


@pytest.mark.parametrize("N", [3, 4])
def test_blast_rhs_nan_pattern(oracle, N):
    """Where the interpolated large-face state is inadmissible both sides leave the
    high-order residual undefined at the same nodes; the low-order residual agrees."""
    spec = random_mesh(10, 8, 2, 0.45, L=4.0, x0=-2.0, y0=-2.0)
    s, M = pair(oracle, spec, N)
    x, y, m = M.geometry()
    u = states.sedov_tophat(x, y, r0=0.5)
    s.upload(u)
    w0 = oracle.basis(N)[1][0]
    for which in (1, 0):
        err = rate_err(s.rhs(which), M.rhs(u, which), u, x, y, w0)
        print(f"blast rhs N={N} which={which} err={err:.2e}", flush=True)
        assert err < TOL


def test_isentropic_near_vacuum_parity(oracle):
    """gamma = 3 near vacuum, low-order time step: limiter active, mortars fall back."""
    import paper_2607_06045_amd as P
    s2 = np.sqrt(2.0)
    spec = refined_box_mesh(8, (-1 / s2, -1 / s2), (0.0, 1 / s2), -s2, -s2, 2 * s2)
    s, M = pair(oracle, spec, 3, gamma=3.0, dt_mode=P.DT_LOWORDER)
    x, y, m = M.geometry()
    u = states.isentropic_flow(x, y, gamma=3.0)
    s.upload(u)
    c = u
    for k in range(3):
        st = s.step(0.5)
        c, sc = M.ssprk3(c, 0.5, mode=oracle.DT_LOWORDER, gamma=3.0)
        err = state_err(s.download(), c, gamma=3.0)
        print(f"isentropic step {k} err={err:.2e} gpu={st}", flush=True)
        assert err < TOL
        assert st["violations"] == 0 and st["fv_inadmissible"] == 0


def test_vortex304_step_parity_and_determinism(oracle):
    """Workload 1: one RHS and one SSP-RK3 step at CFL 0.5; a rerun is bitwise equal."""
    spec = workload_mesh("vortex304")
    s, M = pair(oracle, spec, 3)
    x, y, m = M.geometry()
    u = states.workload_state("vortex304", x, y)
    s.upload(u)
    st = s.step(0.5)
    g1 = s.download()
    c, sc = M.ssprk3(u, 0.5)
    err = state_err(g1, c)
    print(f"vortex304 step err={err:.2e}", flush=True)
    assert err < TOL
    s.upload(u)
    s.step(0.5)
    assert np.array_equal(s.download(), g1)


@pytest.mark.parametrize("k", ["blast22k", "shear59k"])
def test_full_size_workload_step(oracle, k):
    """The blast and shear-layer workloads at full size (22,156 and 59,392 leaves): one SSP-RK3 step
    compared with the oracle on every node."""
    spec = workload_mesh(k)
    s, M = pair(oracle, spec, 3)
    x, y, m = M.geometry()
    u = states.workload_state(k, x, y)
    s.upload(u)
    st = s.step(0.5)
    c, sc = M.ssprk3(u, 0.5)
    err = state_err(s.download(), c)
    print(f"{k} E={s.E} M={s.M} err={err:.2e} gpu={st} oracle={sc}", flush=True)
    assert err < TOL
    assert st["violations"] == 0


def test_error_paths(oracle):
    import paper_2607_06045_amd as P
    s = P.Solver(3)
    spec = workload_mesh("vortex304")
    with pytest.raises(P.DgidpError, match="NO_STATE|NO_MESH"):
        s.step(0.5)
    # unbalanced mesh: a level-2 leaf next to a level-0 leaf
    lv = np.array([0, 0, 0, 1, 1, 1, 2, 2, 2, 2], dtype=np.int8)
    ix = np.array([0, 0, 1, 2, 3, 3, 4, 5, 4, 5], dtype=np.int32)
    iy = np.array([0, 1, 1, 0, 0, 1, 2, 2, 3, 3], dtype=np.int32)
    with pytest.raises(P.DgidpError):
        s.set_mesh(lv, ix, iy, 0.0, 0.0, 1.0, 1.0, 2, 2)
    s.set_mesh(*spec.args())
    x, y = s.node_coords()
    u = states.vortex(x, y)
    u[5, 0, 1, 1] = -1.0
    with pytest.raises(P.DgidpError, match="INADMISSIBLE"):
        s.upload(u)


def test_graph_replay_matches_eager():
    """Enqueue-only steps replay a captured graph: ten replays (alternating the
    two captured graphs), interleaved with an eager step that returns
    statistics and with limited forward-Euler steps (which move the state to
    another buffer), give bit-identical states to kernel-by-kernel launches."""
    import paper_2607_06045_amd as P
    spec = workload_mesh("blast22k")
    out = []
    for graphs in (True, False):
        s = P.Solver(3)
        s.set_graphs(graphs)
        s.set_mesh(*spec.args())
        x, y = s.node_coords()
        s.upload(states.workload_state("blast22k", x, y))
        for k in range(10):
            s.step(0.5, stats=False)
            if k == 4:
                st = s.step(0.5)  # eager, with statistics
                assert st["violations"] == 0
                s.synchronize()
            if k in (6, 7):
                s.limit(2e-6, stats=False)
        out.append(s.download())
    print(f"graph vs eager: max |diff| {np.abs(out[0] - out[1]).max():.3e}", flush=True)
    assert np.array_equal(out[0], out[1])


@pytest.mark.parametrize("N", [3, 4])
def test_degenerate_meshes_parity(oracle, N):
    """A single leaf that is its own neighbour across every face, a 1 x 2 root,
    and a refined 1 x 1 root whose mortars wrap around the periodic box."""
    from workloads.meshes import to_spec
    cases = {"single": to_spec((0.0, 0.0, 1.0, 1.0, 1, 1), {(0, 0, 0)}),
             "two": to_spec((0.0, 0.0, 2.0, 1.0, 2, 1), {(0, 0, 0), (0, 1, 0)}),
             "wrap": to_spec((0.0, 0.0, 1.0, 1.0, 1, 1),
                             {(1, 0, 0), (1, 1, 0), (1, 0, 1), (2, 2, 2), (2, 3, 2), (2, 2, 3), (2, 3, 3)})}
    for name, spec in cases.items():
        s, M = pair(oracle, spec, N)
        x, y, m = M.geometry()
        u = states.density_wave(x, y)
        s.upload(u)
        w0 = oracle.basis(N)[1][0]
        for which in (0, 1):
            err = rate_err(s.rhs(which), M.rhs(u, which), u, x, y, w0)
            assert err < TOL, (name, which, err)
        st = s.step(0.5)
        c, _ = M.ssprk3(u, 0.5)
        err = state_err(s.download(), c)
        print(f"{name} N={N}: E={s.E} M={s.M} step err={err:.2e}", flush=True)
        assert err < TOL and st["violations"] == 0


def test_full_size_quadrants247k_n4(oracle):
    """The largest workload (N = 4, 246,736 leaves, 6.2 M nodes, 5,536
    mortars): one SSP-RK3 step compared with the oracle on every node."""
    spec = workload_mesh("quadrants247k")
    s, M = pair(oracle, spec, 4)
    x, y, m = M.geometry()
    u = states.workload_state("quadrants247k", x, y)
    s.upload(u)
    st = s.step(0.5)
    c, sc = M.ssprk3(u, 0.5)
    err = state_err(s.download(), c)
    print(f"quadrants247k N=4 E={s.E} M={s.M} err={err:.2e} dt gpu {st['dt']!r} oracle {sc['dt']!r}", flush=True)
    assert err < TOL
    assert st["violations"] == 0
    assert abs(st["dt"] - sc["dt"]) <= 1e-14 * sc["dt"]


def test_full_size_quadrants247k_rhs(oracle):
    """The same workload's high- and low-order residuals on every node.  At this
    size (49,348 element batches, 7% of them holding a mortar element) a stage
    is two launches of the element kernel, one over the mortar batches and one
    over the others, and so is the residual."""
    spec = workload_mesh("quadrants247k")
    s, M = pair(oracle, spec, 4)
    x, y, m = M.geometry()
    u = states.workload_state("quadrants247k", x, y)
    s.upload(u)
    w0 = oracle.basis(4)[1][0]
    for which in (0, 1):
        err = rate_err(s.rhs(which), M.rhs(u, which), u, x, y, w0)
        print(f"quadrants247k N=4 rhs which={which} err={err:.2e}", flush=True)
        assert err < TOL


def test_full_size_quadrants247k_mixed(oracle):
    """The two launches of a stage in the mixed mode: one SSP-RK3 step on every
    node against the FP64 oracle, within the FP32 error bound of the mixed
    path (2 (N+1) 20 2^-24 of the flux scale per unit time, 3 CFL of it per
    step), no violations."""
    import paper_2607_06045_amd as P
    spec = workload_mesh("quadrants247k")
    s, M = pair(oracle, spec, 4, precision=P.MIXED)
    x, y, m = M.geometry()
    u = states.workload_state("quadrants247k", x, y)
    s.upload(u)
    st = s.step(0.5)
    c, sc = M.ssprk3(u, 0.5)
    err = state_err(s.download(), c)
    bound = 3 * 0.5 * 2 * 5 * 20 * 2.0 ** -24
    print(f"quadrants247k N=4 mixed err={err:.2e} bound={bound:.2e}", flush=True)
    assert 0.0 < err < bound
    assert st["violations"] == 0
    assert abs(st["dt"] - sc["dt"]) <= 1e-14 * sc["dt"]


@pytest.mark.parametrize("on_device", [False, True])
def test_state_upload_rejects_inadmissible(on_device):
    """Upload from host memory and from a device tensor: a NaN density, an
    infinite energy and a negative pressure are each rejected with the first bad
    node (element, node) in the message, and a rejected upload leaves the
    previous state in place."""
    import torch
    import paper_2607_06045_amd as P
    spec = workload_mesh("vortex304")
    s = P.Solver(3)
    s.set_mesh(*spec.args())
    x, y = s.node_coords()
    good = states.vortex(x, y)
    s.upload(good)
    for v, j, i, val in ((0, 1, 2, np.nan), (3, 0, 3, np.inf), (3, 2, 1, 0.0)):
        u = good.copy()
        u[40, v, j, i] = val
        u[90, 0, 0, 0] = -1.0  # a later bad node: the first one is reported
        arg = torch.from_numpy(u).cuda() if on_device else u
        with pytest.raises(P.DgidpError, match=f"INADMISSIBLE.*element 40 node {j * 4 + i}"):
            s.upload(arg)
        assert np.array_equal(s.download(), good)
