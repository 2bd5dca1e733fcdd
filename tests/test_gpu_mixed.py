"""Mixed precision (FP32 volume flux differencing, FP32 mortar interpolation and
projection, FP64 bounds, limiter and update) against the FP64 oracle.

Parity unpinned by the paper: the paper fixes no mixed-precision result, so the
mixed path is held to an error bound derived from FP32 rounding.  A high-order
residual at a node is a sum of 2(N+1) two-point flux terms (each direction:
N+1 pair terms plus the surface term); each FP32 term carries at most about 20
roundings of unit 2^-24 relative to its own size.  So the residual error is
bounded by TOL_RATE(N) = 2(N+1) * 20 * 2^-24 of the flux-term scale used by
tests/parity.py.  One SSP-RK3 step at CFL c moves a node by at most about
3 c times that scale, so states are held to 3 c TOL_RATE(N).
"""
import numpy as np
import pytest

from parity import rate_err, state_err
from workloads import states
from workloads.meshes import workload_mesh, random_mesh

pytestmark = pytest.mark.gpu


def tol_rate(N):
    return 2 * (N + 1) * 20 * 2.0 ** -24


def solver(spec, N, precision, **kw):
    import paper_2607_06045_amd as P
    s = P.Solver(N, precision=precision, **kw)
    s.set_mesh(*spec.args())
    return s


@pytest.mark.parametrize("N", [3, 4])
@pytest.mark.parametrize("name", ["vortex304", "random3"])
def test_mixed_rhs_error_bound(oracle, name, N):
    import paper_2607_06045_amd as P
    spec = workload_mesh("vortex304") if name == "vortex304" else random_mesh(3, 4, 3, 0.4)
    M = oracle.Mesh(N, *spec.args())
    x, y, m = M.geometry()
    u = states.vortex(x, y) if name == "vortex304" else states.density_wave(x, y)
    s = solver(spec, N, P.MIXED)
    s.upload(u)
    w0 = oracle.basis(N)[1][0]
    for which in (0, 1):
        g = s.rhs(which)
        c = M.rhs(u, which)
        err = rate_err(g, c, u, x, y, w0)
        print(f"mixed rhs {name} N={N} which={which} err={err:.2e} bound={tol_rate(N):.2e}", flush=True)
        if which == 1:
            # the low-order residual is FP64 in both modes
            assert err < 1e-12
        else:
            assert err < tol_rate(N)
            assert err > 0.0  # the FP32 path is really taken


@pytest.mark.parametrize("N", [3, 4])
def test_mixed_step_error_bound(oracle, N):
    import paper_2607_06045_amd as P
    spec = workload_mesh("vortex304")
    M = oracle.Mesh(N, *spec.args())
    x, y, m = M.geometry()
    u = states.workload_state("vortex304", x, y)
    s = solver(spec, N, P.MIXED)
    s.upload(u)
    cfl = 0.5
    st = s.step(cfl)
    ref, _ = M.ssprk3(u, cfl)
    err = state_err(s.download(), ref)
    bound = 3 * cfl * tol_rate(N)
    print(f"mixed step N={N} err={err:.2e} bound={bound:.2e} violations={st['violations']}", flush=True)
    assert st["violations"] == 0
    assert err < bound


def _defect(u0, u1, m):
    """|sum_i m_i (u1 - u0)_i| / sum_i m_i |u0_i|, worst variable."""
    num = np.abs((m[:, None] * (u1 - u0)).sum(axis=(0, 2, 3)))
    den = (m[:, None] * np.abs(u0)).sum(axis=(0, 2, 3))
    return (num / den).max()


def test_mixed_conservation_defect(oracle):
    """FP32 flux differencing stays conservative to FP64 round-off (every
    subcell flux is added to one node and taken from its neighbour, summed in
    FP64); only the FP32 mortar projection leaves a defect, of FP32 size."""
    import paper_2607_06045_amd as P
    out = {}
    for name, spec in (("uniform", random_mesh(5, 12, 0, 0.0)), ("vortex304", workload_mesh("vortex304"))):
        M = oracle.Mesh(3, *spec.args())
        x, y, m = M.geometry()
        u = states.vortex(x, y) if name == "uniform" else states.workload_state("vortex304", x, y)
        for prec in (P.FP64, P.MIXED):
            s = solver(spec, 3, prec)
            s.upload(u)
            s.step(0.5)
            out[name, prec] = _defect(u, s.download(), m)
    print("conservation defect " + ", ".join(f"{k[0]}/{'mixed' if k[1] else 'fp64'} {v:.2e}"
                                              for k, v in out.items()), flush=True)
    assert out["uniform", P.FP64] < 1e-14 and out["vortex304", P.FP64] < 1e-14
    assert out["uniform", P.MIXED] < 1e-14
    assert out["vortex304", P.MIXED] < 2.0 ** -24


def test_mixed_blast_positivity():
    """Limiting in FP64 keeps the bounds exactly in the mixed mode: the full
    benchmark blast for several steps, zero violations, and the mixed solution
    stays close to the FP64 one."""
    import paper_2607_06045_amd as P
    spec = workload_mesh("blast22k")
    res = {}
    for prec in (P.FP64, P.MIXED):
        s = solver(spec, 3, prec)
        x, y = s.node_coords()
        s.upload(states.workload_state("blast22k", x, y))
        viol = inad = 0
        for _ in range(5):
            st = s.step(0.5)
            viol += st["violations"]
            inad += st["fv_inadmissible"]
        res[prec] = (s.download(), viol, inad)
    (u64, v64, i64), (umx, vmx, imx) = res[P.FP64], res[P.MIXED]
    rel_l1 = np.abs(umx - u64).sum(axis=(0, 2, 3)) / np.abs(u64).sum(axis=(0, 2, 3))
    print(f"blast 5 steps: violations fp64 {v64} mixed {vmx}; rel L1 diff {rel_l1}", flush=True)
    assert v64 == 0 and vmx == 0 and i64 == 0 and imx == 0
    assert rel_l1.max() < 1e-5
