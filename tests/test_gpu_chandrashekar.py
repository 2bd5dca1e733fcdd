"""GPU volume flux differencing with the Chandrashekar flux (Sec. 3.6) against the
oracle, through the C-ABI: residuals, a limited step, and a blast run."""
import numpy as np
import pytest

from parity import rate_err, state_err
from workloads import states
from workloads.meshes import random_mesh

pytestmark = pytest.mark.gpu
TOL = 1e-12


def pair(oracle, spec, N=3, **kw):
    import paper_2607_06045_amd as P
    s = P.Solver(N, volume_flux=P.FLUX_CHANDRASHEKAR, **kw)
    s.set_mesh(*spec.args())
    M = oracle.Mesh(N, *spec.args(), volume_flux="chandrashekar")
    assert (s.E, s.M) == (M.E, M.M)
    return s, M


@pytest.mark.parametrize("N", [3, 4])
def test_chandrashekar_rhs_parity(oracle, N):
    s, M = pair(oracle, random_mesh(3, 4, 3, 0.4), N)
    x, y, m = M.geometry()
    u = states.random_admissible(x, 9, rho_range=(0.8, 1.2), p_range=(0.8, 1.2), vmax=0.3)
    s.upload(u)
    w0 = oracle.basis(N)[1][0]
    g = s.rhs(0)
    c = M.rhs(u, oracle.RHS_HIGH)
    err = rate_err(g, c, u, x, y, w0)
    print(f"chandrashekar rhs N={N} err={err:.2e}", flush=True)
    assert err < TOL
    # a different scheme from the default flux
    import paper_2607_06045_amd as P
    r = P.Solver(N)
    r.set_mesh(*random_mesh(3, 4, 3, 0.4).args())
    r.upload(u)
    assert np.abs(r.rhs(0) - g).max() > 1e-6 * np.abs(g).max()


@pytest.mark.parametrize("N", [3, 4])
def test_chandrashekar_blast_steps_parity(oracle, N):
    """Top-hat blast with positivity limiting and mortars, three SSP-RK3 steps."""
    spec = random_mesh(10, 8, 2, 0.45, L=4.0, x0=-2.0, y0=-2.0)
    s, M = pair(oracle, spec, N)
    x, y, m = M.geometry()
    u = states.sedov_tophat(x, y, r0=0.5)
    s.upload(u)
    c = u
    for k in range(3):
        st = s.step(0.9)
        c, sc = M.ssprk3(c, 0.9)
        err = state_err(s.download(), c)
        print(f"chandrashekar blast N={N} step {k} err={err:.2e}", flush=True)
        assert err < TOL
        assert st["violations"] == 0
        assert abs(st["dt"] - sc["dt"]) <= 1e-13 * sc["dt"]
