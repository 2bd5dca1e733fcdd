"""Host logic of mesh adaptation in the GPU library against the oracle
(integer work: bit-exact), and the three-level controller."""
import numpy as np
import pytest

from workloads.meshes import workload_mesh, random_flags, random_mesh


@pytest.mark.parametrize("seed", range(8))
def test_adapt_leaves_matches_oracle(oracle, seed):
    import paper_2607_06045_amd as P
    spec = random_mesh(seed, 4 + seed % 3, 3, 0.4)
    flags = random_flags(spec, 50 + seed, p_refine=0.1 + 0.03 * seed, p_coarsen=0.6)
    a = P.adapt_leaves(spec.level, spec.ix, spec.iy, spec.nx0, spec.ny0, flags)
    b = oracle.adapt(spec.level, spec.ix, spec.iy, spec.nx0, spec.ny0, flags)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)
    # the result is a valid balanced mesh for the library too
    P.validate_mesh(3, a[0], a[1], a[2], spec.nx0, spec.ny0)


@pytest.mark.parametrize("k", ["vortex304", "blast22k"])
def test_adapt_leaves_workloads(oracle, k):
    import paper_2607_06045_amd as P
    spec = workload_mesh(k)
    flags = random_flags(spec, 9, p_refine=0.05, p_coarsen=0.5)
    a = P.adapt_leaves(spec.level, spec.ix, spec.iy, spec.nx0, spec.ny0, flags)
    b = oracle.adapt(spec.level, spec.ix, spec.iy, spec.nx0, spec.ny0, flags)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


def test_adapt_leaves_errors():
    import paper_2607_06045_amd as P
    spec = random_mesh(1, 4, 1, 0.3)
    with pytest.raises(P.DgidpError):
        P.adapt_leaves(spec.level, spec.ix, spec.iy, 0, spec.ny0, np.zeros(spec.E, np.int8))


def test_amr_flags_three_levels():
    import paper_2607_06045_amd as P
    ind = np.array([0.0, 0.2, 0.6, 0.9, 0.9, 0.0, 0.6], np.float32)
    lev = np.array([6, 6, 6, 6, 9, 8, 8], np.int8)
    f = P.amr_flags(ind, lev, base_level=6, med_level=7, med_threshold=0.5, max_level=9,
                    max_threshold=0.8)
    assert f.tolist() == [0, 0, 1, 1, 0, -1, -1]
    with pytest.raises(P.DgidpError):
        P.amr_flags(ind, lev, 6, 5, 0.5, 9, 0.8)
