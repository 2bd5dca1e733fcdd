"""GPU mortar limiter at fractional factors (Sec. 2.3, Mortar Limiting; positivity
bounds of eq. Bounds_Positivity) against the oracle, through the C-ABI.

The cases are those of test_oracle_mortar.py, where the oracle's factors are
pinned to a brute-force scan: strict bounds (beta = 0.999 and 0.99) on smooth
states, which make every or nearly every mortar factor fractional, including
mortars whose binding node lies on two mortars (L-shaped refinement), and two
blasts at the paper's beta = 0.1 with a fractional factor.  One limited
forward-Euler step and one SSP-RK3 step are compared node by node at 1e-12
(the state metric of parity.py), the smallest and the mean mortar factor at
1e-10, and the smallest factor is required to lie strictly between 0 and 1
where no mortar of the case falls back to the low-order flux."""
import numpy as np
import pytest

from parity import state_err
from test_oracle_mortar import CASES, IDS

pytestmark = pytest.mark.gpu
TOL = 1e-12


@pytest.mark.parametrize("case", range(len(CASES)), ids=IDS)
def test_fractional_mortar_factor_parity(oracle, case):
    import paper_2607_06045_amd as P
    N, spec, u, cfl, beta = CASES[case]
    M = oracle.Mesh(N, *spec.args())
    s = P.Solver(N, beta=beta)
    s.set_mesh(*spec.args())
    s.upload(u)
    dt = M.max_dt(u, cfl)
    st = s.limit(dt)
    c, sc, uvol, dslot, theta = M.fe_step_detail(u, dt, beta=beta)
    err = state_err(s.download(), c)
    print(f"mortar FE {IDS[case]} err={err:.2e} theta_mort_min gpu={st['theta_mort_min']!r} "
          f"oracle={sc['theta_mort_min']!r}", flush=True)
    assert err < TOL
    assert st["violations"] == 0 and sc["violations"] == 0
    assert abs(st["theta_mort_min"] - sc["theta_mort_min"]) < 1e-10
    assert abs(st["alpha_mort_mean"] - sc["alpha_mort_mean"]) < 1e-10
    # the step has fractional mortar factors; where no mortar falls back to the
    # low-order flux (factor 0) the smallest one is fractional
    assert np.any((theta > 0.0) & (theta < 1.0))
    if np.all(theta > 0.0):
        assert 0.0 < st["theta_mort_min"] < 1.0
    # one SSP-RK3 step from the same state
    s.upload(u)
    stp = s.step(cfl)
    ref, sref = M.ssprk3(u, cfl, beta=beta)
    err = state_err(s.download(), ref)
    print(f"mortar step {IDS[case]} err={err:.2e} dt={stp['dt']!r}", flush=True)
    assert abs(stp["dt"] - sref["dt"]) <= 1e-13 * sref["dt"]
    assert err < TOL
    assert stp["violations"] == 0
    assert abs(stp["theta_mort_min"] - sref["theta_mort_min"]) < 1e-10
