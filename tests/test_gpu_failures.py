"""Failure detection and recovery through the C-ABI (GPU): the time-step guard of
strict mode, positivity loss without the limiter against none with it, the
detection of inadmissible (NaN) states, checkpoint and resume, and an
adaptation beyond the kernels' size limit that keeps mesh and state.

The method's own failure mode is a state outside the admissible set (rho <= 0
or p <= 0), which the IDP limiter prevents (Sec. 2.2-2.3; the Sedov blast of
Sec. 3.4 is the paper's positivity test)."""
import numpy as np
import pytest

from workloads import states
from workloads.meshes import random_mesh, workload_mesh

pytestmark = pytest.mark.gpu


def blast(N=3, **kw):
    import paper_2607_06045_amd as P
    spec = random_mesh(10, 8, 2, 0.45, L=4.0, x0=-2.0, y0=-2.0)
    s = P.Solver(N, **kw)
    s.set_mesh(*spec.args())
    x, y = s.node_coords()
    return s, spec, states.sedov_tophat(x, y, r0=0.5)


def test_strict_dt_rejects_a_step_above_the_idp_bound():
    """strict mode: a forward-Euler step above the IDP bound (eq.
    timestep_restriction) returns DGIDP_E_DT and leaves the state untouched;
    at the bound it is taken"""
    import paper_2607_06045_amd as P
    s, spec, u = blast(strict_dt=True)
    s.upload(u)
    bound = s.max_dt(1.0)
    with pytest.raises(P.DgidpError, match="E_DT"):
        s.limit(bound * 1.001)
    assert np.array_equal(s.download(), u)
    st = s.limit(bound)
    assert st["violations"] == 0 and st["fv_inadmissible"] == 0
    # without strict mode the same call is taken
    s2, _, _ = blast()
    s2.upload(u)
    s2.limit(bound * 1.001)


def test_limiter_off_loses_positivity_limiter_on_keeps_it(oracle):
    """Top-hat blast (p = 1e-5 outside): without the limiter the high-order
    steps leave the positivity bounds rho >= 0.1 rho^FV, p >= 0.1 p^FV and soon
    the admissible set; with positivity limiting no bound is violated"""
    import paper_2607_06045_amd as P
    N = 3
    M = None
    for limiter in (P.LIMIT_NONE, P.LIMIT_POSITIVITY):
        s, spec, u = blast(N, limiter=limiter)
        if M is None:
            M = oracle.Mesh(N, *spec.args())
        s.upload(u)
        viol, inad = 0, 0
        w = u
        for k in range(5):
            dt = M.max_dt(w, 0.5)
            st = s.limit(dt)
            new = s.download()
            # the positivity bounds of this step from the oracle's low-order state
            ufv = w + dt * M.rhs(w, oracle.RHS_LOW)
            rho, p = new[:, 0], (0.4 * (new[:, 3] - 0.5 * (new[:, 1] ** 2 + new[:, 2] ** 2) / new[:, 0]))
            pfv = 0.4 * (ufv[:, 3] - 0.5 * (ufv[:, 1] ** 2 + ufv[:, 2] ** 2) / ufv[:, 0])
            bad = ~(rho >= 0.1 * ufv[:, 0]) | ~(p >= 0.1 * pfv)
            viol += int(bad.sum())
            inad += int((~(rho > 0) | ~(p > 0)).sum())
            print(f"limiter={limiter} step {k}: bound violations {int(bad.sum())}, "
                  f"inadmissible {int((~(rho > 0) | ~(p > 0)).sum())}, gpu stats {st}", flush=True)
            if limiter == P.LIMIT_POSITIVITY:
                assert st["violations"] == 0
            if inad:
                break
            w = new
        if limiter == P.LIMIT_NONE:
            assert viol > 0 and inad > 0
        else:
            assert viol == 0 and inad == 0


def test_inadmissible_state_is_detected():
    """An unlimited blast runs out of the admissible set: the step statistics
    report inadmissible low-order states once the state holds a NaN or a
    negative pressure, and dgidp_state_check names a bad node, which the
    downloaded state confirms; the limited run reports none"""
    import paper_2607_06045_amd as P
    s, spec, u = blast(limiter=P.LIMIT_NONE)
    s.upload(u)
    assert s.check_state() is None
    found = None
    for k in range(40):
        s.step(0.5, stats=False)
        found = s.check_state()
        if found is not None:
            break
    assert found is not None, "the unlimited blast stayed admissible"
    e, q = found
    w = s.download()[e].reshape(4, -1)[:, q]
    p = 0.4 * (w[3] - 0.5 * (w[1] ** 2 + w[2] ** 2) / w[0])
    print(f"unlimited blast: inadmissible after {k + 1} steps at element {e} node {q}: {w}, p={p}", flush=True)
    assert not (np.all(np.isfinite(w)) and w[0] > 0 and p > 0)
    st = s.step(0.5)
    assert st["fv_inadmissible"] > 0
    # the state cannot be re-uploaded as it is
    with pytest.raises(P.DgidpError, match="INADMISSIBLE"):
        s.upload(s.download())
    s2, _, _ = blast()
    s2.upload(u)
    for _ in range(k + 2):
        st2 = s2.step(0.5)
        assert st2["fv_inadmissible"] == 0 and st2["violations"] == 0
    assert s2.check_state() is None


def test_checkpoint_resume_is_bitwise():
    """k steps, an adaptation, more steps; download mesh and state, build a new
    context from them and continue: bitwise equal to the uninterrupted run"""
    import paper_2607_06045_amd as P
    spec = workload_mesh("vortex304")

    def fresh():
        s = P.Solver(3)
        s.set_mesh(*spec.args())
        return s

    s = fresh()
    x, y = s.node_coords()
    s.upload(states.vortex(x, y))
    for _ in range(3):
        s.step(0.5, stats=False)
    flags = np.zeros(s.E, dtype=np.int8)
    flags[::7] = 1
    s.refine_coarsen(flags)
    for _ in range(2):
        s.step(0.5, stats=False)
    level, ix, iy = s.mesh()
    ck = s.download()
    # resume in a new context
    r = P.Solver(3)
    r.set_mesh(level, ix, iy, spec.x0, spec.y0, spec.Lx, spec.Ly, spec.nx0, spec.ny0)
    r.upload(ck)
    assert np.array_equal(r.download(), ck)
    for _ in range(4):
        s.step(0.5, stats=False)
        r.step(0.5, stats=False)
    a, b = s.download(), r.download()
    print(f"resume: max |diff| {np.abs(a - b).max():.3e}", flush=True)
    assert np.array_equal(a, b)


def test_adaptation_beyond_the_size_limit_keeps_mesh_and_state():
    """An adaptation whose new leaf count exceeds the kernels' index range
    (2^30 / (4 (N+1)^2) leaves) is refused with DGIDP_E_INVALID_ARG before the
    current mesh and state are let go; the context keeps stepping"""
    import paper_2607_06045_amd as P
    N = 4
    limit = (1 << 30) // (4 * (N + 1) ** 2)          # 10,737,418 leaves
    nx0 = ny0 = 1639                                  # 2,686,321 leaves; refined: above the limit
    assert nx0 * ny0 <= limit < 4 * nx0 * ny0
    lev = np.zeros(nx0 * ny0, dtype=np.int8)
    ix = np.tile(np.arange(nx0, dtype=np.int32), ny0)
    iy = np.repeat(np.arange(ny0, dtype=np.int32), nx0)
    s = P.Solver(N)
    s.set_mesh(lev, ix, iy, 0.0, 0.0, 1.0, 1.0, nx0, ny0)
    x, y = s.node_coords()
    u = states.conservative(1.0 + 0.1 * np.sin(2 * np.pi * x), 0.5 + 0 * x, 0 * x, 1.0 + 0 * x, 1.4)
    del x, y
    s.upload(u)
    with pytest.raises(P.DgidpError, match="INVALID_ARG"):
        s.refine_coarsen(np.ones(s.E, dtype=np.int8))
    assert s.E == nx0 * ny0
    assert np.array_equal(s.download(), u)
    st = s.step(0.5)
    assert st["violations"] == 0
