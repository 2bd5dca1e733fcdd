"""Seeded synthetic inputs: mesh sizes of the named workloads, 2:1 balance,
RNG determinism, admissible initial states."""
import numpy as np
import pytest

from workloads import rng, states
from workloads.meshes import workload_mesh, random_mesh


def test_splitmix64_reference_values():
    # SplitMix64 with state 0: first outputs of the published generator
    z = rng.splitmix64(0, np.arange(3, dtype=np.uint64))
    assert [int(v) for v in z] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]
    u = rng.uniform(7, np.arange(1000, dtype=np.uint64))
    assert (u >= 0).all() and (u < 1).all() and abs(u.mean() - 0.5) < 0.03


@pytest.mark.parametrize("k,E,levels", [
    ("vortex304", 304, {0: 240, 1: 64}),
    ("blast22k", 22156, {0: 3744, 1: 176, 2: 492, 3: 17744}),
    ("shear59k", 59392, {0: 15360, 1: 1024, 2: 2048, 3: 40960}),
])
def test_workload_meshes(oracle, k, E, levels):
    m = workload_mesh(k)
    assert m.E == E and m.counts() == levels
    M = oracle.Mesh(3, *m.args())  # tiles the domain and is 2:1 balanced
    assert M.E == E


def test_workload_states_admissible(oracle):
    for k in ("vortex304", "blast22k", "shear59k"):
        M = oracle.Mesh(3, *workload_mesh(k).args())
        x, y, m = M.geometry()
        u = states.workload_state(k, x, y)
        p = 0.4 * (u[:, 3] - 0.5 * (u[:, 1] ** 2 + u[:, 2] ** 2) / u[:, 0])
        assert (u[:, 0] > 0).all() and (p > 0).all()


def test_random_mesh_deterministic():
    a, b = random_mesh(4, 4, 3, 0.4), random_mesh(4, 4, 3, 0.4)
    assert np.array_equal(a.level, b.level) and np.array_equal(a.ix, b.ix)
