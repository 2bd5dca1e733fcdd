"""GPU combined limiting (Sec. 3.5, eq. combination_posLim_local) against the
oracle, through the C-ABI: per subcell face alpha = (1 - w) alpha_pos +
w alpha_local, w the element's shock indicator on the pressure."""
import numpy as np
import pytest

from parity import state_err
from workloads import states
from workloads.meshes import random_mesh, workload_mesh

pytestmark = pytest.mark.gpu
TOL = 1e-12


def pair(oracle, spec, N=3, limiter=None, **kw):
    import paper_2607_06045_amd as P
    s = P.Solver(N, limiter=P.LIMIT_COMBINED if limiter is None else limiter, **kw)
    s.set_mesh(*spec.args())
    M = oracle.Mesh(N, *spec.args())
    assert (s.E, s.M) == (M.E, M.M)
    return s, M


BLAST = lambda: random_mesh(10, 8, 2, 0.45, L=4.0, x0=-2.0, y0=-2.0)  # noqa: E731


@pytest.mark.parametrize("N", [3, 4])
def test_combined_stages_parity(oracle, N):
    """Top-hat blast: the indicator marks the shock elements, which get the local
    factors, the rest the positivity factors.  Each SSP-RK3 stage of two steps is
    one limited forward-Euler step of the GPU on the oracle's stage input (the
    local factors amplify rounding on this flow as for pure local limiting, so
    the bound is 1e-10)."""
    s, M = pair(oracle, BLAST(), N)
    x, y, m = M.geometry()
    c = states.sedov_tophat(x, y, r0=0.5)
    w = M.shock_indicator(c)
    assert 0 < (w > 0).sum() < M.E
    worst = 0.0
    for k in range(2):
        dt = M.max_dt(c, 0.9)
        stage_in = c
        for a_, b_ in ((0.0, 1.0), (0.75, 0.25), (1.0 / 3.0, 2.0 / 3.0)):
            s.upload(stage_in)
            st = s.limit(dt)
            wst, sw = M.fe_step(stage_in, dt, limiter=oracle.LIM_COMBINED)
            err = state_err(s.download(), wst)
            worst = max(worst, err)
            print(f"  stage err={err:.2e} alpha_vol gpu={st['alpha_vol_mean']:.6f} "
                  f"oracle={sw['alpha_vol_mean']:.6f}", flush=True)
            assert st["violations"] == 0 and sw["violations"] == 0
            stage_in = a_ * c + b_ * wst
        c = stage_in
    print(f"combined blast stages N={N} worst err={worst:.2e}", flush=True)
    assert worst < 1e-10


@pytest.mark.parametrize("N", [3, 4])
def test_combined_forward_euler_parity_random(oracle, N):
    """Random states on a mesh with mortars: every face and mortar blends the two
    factor sets (at N = 3 the indicator takes values inside (0, 1); at N = 4 its
    threshold is lower and it is 1 on these states)."""
    s, M = pair(oracle, random_mesh(0, 4, 3, 0.4), N)
    x, y, m = M.geometry()
    u = states.random_admissible(x, 11, rho_range=(0.5, 1.5), p_range=(0.5, 1.5), vmax=0.5)
    w = M.shock_indicator(u)
    assert (w > 0).any() and (N == 4 or ((w > 0) & (w < 1)).any())
    s.upload(u)
    dt = M.max_dt(u, 0.9)
    st = s.limit(dt)
    c, sc = M.fe_step(u, dt, limiter=oracle.LIM_COMBINED)
    err = state_err(s.download(), c)
    print(f"combined fe random N={N} err={err:.2e} gpu={st} oracle={sc}", flush=True)
    assert err < TOL
    assert st["violations"] == 0
    assert abs(st["alpha_vol_mean"] - sc["alpha_vol_mean"]) < 1e-10
    assert abs(st["alpha_mort_mean"] - sc["alpha_mort_mean"]) < 1e-10


def test_combined_is_positivity_where_smooth():
    """A density wave has constant pressure, so the indicator is 0 everywhere and
    combined limiting is the positivity-limited scheme (to rounding: the two
    kernel variants are compiled separately, 1e-14 apart after five steps)."""
    import paper_2607_06045_amd as P
    spec = random_mesh(3, 4, 3, 0.4)
    out = []
    for lim in (P.LIMIT_COMBINED, P.LIMIT_POSITIVITY):
        s = P.Solver(3, limiter=lim)
        s.set_mesh(*spec.args())
        x, y = s.node_coords()
        s.upload(states.density_wave(x, y))
        for _ in range(5):
            s.step(0.9)
        out.append(s.download())
        s.close()
    assert state_err(out[0], out[1]) < 1e-13


def test_combined_blast22k_full_size(oracle):
    """The 22,156-leaf Gaussian blast, one SSP-RK3 step at full size."""
    spec = workload_mesh("blast22k")
    s, M = pair(oracle, spec, 3)
    x, y, m = M.geometry()
    u = states.workload_state("blast22k", x, y)
    s.upload(u)
    st = s.step(0.5)
    c, sc = M.ssprk3(u, 0.5, limiter=oracle.LIM_COMBINED)
    err = state_err(s.download(), c)
    print(f"combined blast22k err={err:.2e} gpu={st} oracle={sc}", flush=True)
    assert err < TOL
    assert st["violations"] == 0 and st["dt"] == sc["dt"]


@pytest.mark.parametrize("N", [3, 4])
def test_combined_blast_run_valid(oracle, N):
    """Three SSP-RK3 steps of the GPU on its own: positivity bounds, conservation,
    and agreement with the oracle's run in the mean."""
    s, M = pair(oracle, BLAST(), N)
    x, y, m = M.geometry()
    u = states.sedov_tophat(x, y, r0=0.5)
    s.upload(u)
    c = u
    tot0 = (u * m[:, None]).sum(axis=(0, 2, 3))
    for k in range(3):
        st = s.step(0.9)
        c, sc = M.ssprk3(c, 0.9, limiter=oracle.LIM_COMBINED)
        assert st["violations"] == 0 and sc["violations"] == 0
    g = s.download()
    tot = (g * m[:, None]).sum(axis=(0, 2, 3))
    scale = (np.abs(g) * m[:, None]).sum(axis=(0, 2, 3))
    assert np.all(np.abs(tot - tot0) < 1e-13 * scale)
    l1 = (np.abs(g - c) * m[:, None]).sum(axis=(0, 2, 3)) / scale
    print(f"combined blast run N={N} rel L1 diff per variable={l1}", flush=True)
    assert l1.max() < 1e-9
