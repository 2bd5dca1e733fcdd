"""The allocation-free SSP-RK3 step (dgidp_step_noalloc) against dgidp_step,
through the C-ABI: the same kernels on buffers carved from the library's static
per-device scratch array, so the states agree bit for bit.  Two calls in a row
on one GPU, the second on a smaller mesh (the array keeps the first call's
contents), for the positivity, combined and low-order-bounds limiters; a mesh
that does not fit is refused before any work is enqueued."""
import numpy as np
import pytest

from workloads import states
from workloads.meshes import random_mesh, workload_mesh

pytestmark = pytest.mark.gpu


def pair(spec, N, x_state, **kw):
    import paper_2607_06045_amd as P
    out = []
    for _ in range(2):
        s = P.Solver(N, **kw)
        s.set_mesh(*spec.args())
        x, y = s.node_coords()
        s.upload(x_state(x, y))
        out.append(s)
    return out


@pytest.mark.parametrize("limiter", ["positivity", "combined", "local_lowsol"])
def test_noalloc_step_matches_step(limiter):
    import paper_2607_06045_amd as P
    kw = {"positivity": {}, "combined": {"limiter": P.LIMIT_COMBINED},
          "local_lowsol": {"limiter": P.LIMIT_LOCAL_LOWORDER, "dt_mode": P.DT_LOWORDER}}[limiter]
    cfl = 0.4 if limiter == "local_lowsol" else 0.5
    big = random_mesh(10, 8, 2, 0.45, L=4.0, x0=-2.0, y0=-2.0)      # blast mesh
    small = workload_mesh("vortex304")
    cases = [(big, 3, lambda x, y: states.sedov_tophat(x, y, r0=0.5)),
             (small, 4, lambda x, y: states.vortex(x, y))]
    solvers = [pair(spec, N, f, **kw) for spec, N, f in cases]
    assert solvers[1][0].E < solvers[0][0].E
    for k in range(3):
        for (ref, nal), (spec, N, _) in zip(solvers, cases):
            ref.step(cfl, stats=False)
            nal.step_noalloc(cfl)
            a, b = ref.download(), nal.download()
            print(f"{limiter} step {k} E={ref.E} N={N}: max |diff| {np.abs(a - b).max():.3e}", flush=True)
            assert np.array_equal(a, b)


def test_noalloc_step_refuses_a_mesh_that_does_not_fit():
    """about 1.0 million nodes fit the 64 MiB array; 512^2 elements at N = 3
    (4.2 million nodes) do not: DGIDP_E_INVALID_ARG, state unchanged"""
    import paper_2607_06045_amd as P
    from workloads.meshes import uniform_mesh
    spec = uniform_mesh(512, 512)
    s = P.Solver(3)
    s.set_mesh(*spec.args())
    x, y = s.node_coords()
    u = states.density_wave(x, y)
    s.upload(u)
    with pytest.raises(P.DgidpError, match="INVALID_ARG"):
        s.step_noalloc(0.5)
    s.synchronize()
    assert np.array_equal(s.download(), u)
