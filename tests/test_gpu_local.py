"""GPU local limiting (eq. Bounds_Barstates) against the oracle, through the C-ABI.

Tolerance: 1e-12 relative per DOF (the state metric of parity.py), FP64 path.
Local limiting is active on smooth data as well (the bar-state bounds are tight),
so every case below exercises the entropy root and the two-sided density factor."""
import numpy as np
import pytest

from parity import state_err
from workloads import states
from workloads.meshes import random_mesh, refined_box_mesh, workload_mesh

pytestmark = pytest.mark.gpu
TOL = 1e-12


def pair(oracle, spec, N=3, **kw):
    import paper_2607_06045_amd as P
    s = P.Solver(N, limiter=P.LIMIT_LOCAL, **kw)
    s.set_mesh(*spec.args())
    M = oracle.Mesh(N, *spec.args())
    assert (s.E, s.M) == (M.E, M.M)
    return s, M


CASES = {
    "random3-density-wave": (lambda: random_mesh(3, 4, 3, 0.4), lambda x, y: states.density_wave(x, y)),
    "random0-random": (lambda: random_mesh(0, 4, 3, 0.4),
                       lambda x, y: states.random_admissible(x, 11, rho_range=(0.5, 1.5),
                                                             p_range=(0.5, 1.5), vmax=0.5)),
    "vortex304": (lambda: workload_mesh("vortex304"), lambda x, y: states.vortex(x, y)),
}


@pytest.mark.parametrize("N", [3, 4])
@pytest.mark.parametrize("name", sorted(CASES))
def test_local_forward_euler_parity(oracle, name, N):
    mesh, init = CASES[name]
    s, M = pair(oracle, mesh(), N)
    x, y, m = M.geometry()
    u = init(x, y)
    s.upload(u)
    dt = M.max_dt(u, 0.9)
    st = s.limit(dt)
    c, sc = M.fe_step(u, dt, limiter=oracle.LIM_LOCAL)
    err = state_err(s.download(), c)
    print(f"local fe {name} N={N} err={err:.2e} gpu={st} oracle={sc}", flush=True)
    assert err < TOL
    assert st["violations"] == 0 and sc["violations"] == 0
    assert abs(st["theta_vol_min"] - sc["theta_vol_min"]) < 1e-10
    assert sc["theta_vol_min"] < 1.0  # the local bounds act


@pytest.mark.parametrize("N", [3, 4])
def test_local_blast_stages_parity(oracle, N):
    """Top-hat blast with mortars: volume and mortar factors, entropy roots at
    shocks, undefined high-order mortar fluxes near vacuum.  Each SSP-RK3 stage of
    two steps is one limited forward-Euler step of the GPU on the oracle's stage
    input, compared node by node.  Local limiting amplifies rounding at some nodes
    of this flow (ambient pressure 1e-5): the oracle's own output moves by up to
    2e-11 under a relative 1e-16 perturbation of its input (printed per stage), so
    the bound here is 1e-10 instead of 1e-12."""
    spec = random_mesh(10, 8, 2, 0.45, L=4.0, x0=-2.0, y0=-2.0)
    s, M = pair(oracle, spec, N)
    x, y, m = M.geometry()
    c = states.sedov_tophat(x, y, r0=0.5)
    rng = np.random.default_rng(5)
    thmin = 1.0
    for k in range(2):
        dt = M.max_dt(c, 0.9)
        stage_in = c
        for a_, b_ in ((0.0, 1.0), (0.75, 0.25), (1.0 / 3.0, 2.0 / 3.0)):
            s.upload(stage_in)
            st = s.limit(dt)
            w, sw = M.fe_step(stage_in, dt, limiter=oracle.LIM_LOCAL)
            err = state_err(s.download(), w)
            sens = 0.0
            for _ in range(2):
                pert = stage_in * (1 + 1e-16 * rng.standard_normal(stage_in.shape))
                sens = max(sens, state_err(M.fe_step(pert, dt, limiter=oracle.LIM_LOCAL)[0], w))
            print(f"local blast N={N} step {k} err={err:.2e} oracle sensitivity={sens:.2e}", flush=True)
            assert err < 1e-10
            assert st["violations"] == 0 and sw["violations"] == 0
            thmin = min(thmin, sw["theta_vol_min"], sw["theta_mort_min"])
            stage_in = a_ * c + b_ * w
        c = stage_in
    assert thmin == 0.0


@pytest.mark.parametrize("N", [3, 4])
def test_local_blast_run_valid(oracle, N):
    """Three SSP-RK3 steps of the GPU on its own: no bound violations, mass,
    momentum and energy conserved, and the state close to the oracle's run.  The
    local factors are discontinuous in the data where a node sits on its bound
    (the paper remarks on this sensitivity for constant regions), so rounding
    differences between the stages of the two runs can flip a factor between 0
    and 1; the runs are compared in the mean (relative L1 per variable)."""
    spec = random_mesh(10, 8, 2, 0.45, L=4.0, x0=-2.0, y0=-2.0)
    s, M = pair(oracle, spec, N)
    x, y, m = M.geometry()
    u = states.sedov_tophat(x, y, r0=0.5)
    s.upload(u)
    c = u
    tot0 = (u * m[:, None]).sum(axis=(0, 2, 3))
    for k in range(3):
        st = s.step(0.9)
        c, sc = M.ssprk3(c, 0.9, limiter=oracle.LIM_LOCAL)
        assert st["violations"] == 0 and sc["violations"] == 0
        assert abs(st["dt"] - sc["dt"]) <= 1e-4 * sc["dt"]
    g = s.download()
    tot = (g * m[:, None]).sum(axis=(0, 2, 3))
    scale = (np.abs(g) * m[:, None]).sum(axis=(0, 2, 3))
    assert np.all(np.abs(tot - tot0) < 1e-13 * scale)
    l1 = (np.abs(g - c) * m[:, None]).sum(axis=(0, 2, 3)) / scale
    print(f"local blast run N={N} rel L1 diff per variable={l1}", flush=True)
    assert l1.max() < 1e-9


def test_local_density_wave_run_parity(oracle):
    """The convergence-test density wave (Sec. 3.1) on the level-2 refined-box
    mesh, 40 steps at CFL 0.95: the limiter cuts the high-order fluxes on the
    smooth wave at every step; states stay within 1e-12 of the oracle."""
    ms = refined_box_mesh(4, (-0.5, -0.5), (0.0, 0.5), -1.0, -1.0, 2.0)
    s, M = pair(oracle, ms, 3)
    x, y, m = M.geometry()
    u = states.density_wave(x, y)
    s.upload(u)
    c = u
    worst = 0.0
    for k in range(40):
        dt = M.max_dt(c, 0.95)
        st = s.step_dt(dt)
        c, sc = M.ssprk3_dt(c, dt, limiter=oracle.LIM_LOCAL)
        worst = max(worst, state_err(s.download(), c))
        assert st["violations"] == 0
    print(f"local density wave 40 steps worst err={worst:.2e} alpha_vol={sc['alpha_vol_mean']:.3f}",
          flush=True)
    assert worst < TOL
    assert sc["alpha_vol_mean"] > 0.01


def test_local_full_size_blast22k(oracle):
    """The 22,156-leaf blast at full size, one SSP-RK3 step, every node."""
    spec = workload_mesh("blast22k")
    s, M = pair(oracle, spec, 3)
    x, y, m = M.geometry()
    u = states.workload_state("blast22k", x, y)
    s.upload(u)
    st = s.step(0.5)
    c, sc = M.ssprk3(u, 0.5, limiter=oracle.LIM_LOCAL)
    err = state_err(s.download(), c)
    print(f"local blast22k err={err:.2e} gpu={st} oracle={sc}", flush=True)
    assert err < TOL
    assert st["violations"] == 0 and st["dt"] == sc["dt"]


def test_local_mixed_precision(oracle):
    """Mixed precision with local limiting: FP32 volume fluxes and mortar
    projection, FP64 bounds, limiter and update.  No bound violations, and mass,
    momentum and energy conserved to the FP32-projection level.  The local
    factors react to the FP32 rounding of the antidiffusive fluxes (a flux of 20
    rounded to FP32 moves f_HO - f_FV by 1e-6 where that difference is 1e-5), so
    the state departs from the FP64 run by far more than FP32 rounding at a few
    nodes (measured: 9e-3 per DOF at worst on the density wave after 10 steps,
    8.7e-6 in relative L1; 2.5e-8 and 1e-7 on the top-hat blast).  The relative
    L1 difference is bounded by 1e-4."""
    import paper_2607_06045_amd as P
    for name, spec, init, steps in (
            ("density wave", random_mesh(3, 4, 3, 0.4), lambda x, y: states.density_wave(x, y), 10),
            ("top-hat blast", random_mesh(10, 8, 2, 0.45, L=4.0, x0=-2.0, y0=-2.0),
             lambda x, y: states.sedov_tophat(x, y, r0=0.5), 3)):
        s, M = pair(oracle, spec, 3, precision=P.MIXED)
        x, y, m = M.geometry()
        c = init(x, y)
        tot0 = (c * m[:, None]).sum(axis=(0, 2, 3))
        s.upload(c)
        for k in range(steps):
            dt = M.max_dt(c, 0.9)
            st = s.step_dt(dt)
            c, sc = M.ssprk3_dt(c, dt, limiter=oracle.LIM_LOCAL)
            assert st["violations"] == 0
        g = s.download()
        scale = (np.abs(g) * m[:, None]).sum(axis=(0, 2, 3))
        cons = np.abs((g * m[:, None]).sum(axis=(0, 2, 3)) - tot0) / scale
        l1 = (np.abs(g - c) * m[:, None]).sum(axis=(0, 2, 3)) / scale
        print(f"local mixed {name}: max err {state_err(g, c):.2e}, rel L1 {l1}, "
              f"conservation {cons}", flush=True)
        assert l1.max() < 1e-4
        assert cons.max() < 1e-9
