"""Pins of the oracle's modal indicator and features (oracle/indicator.py):
closed forms of the orthonormal modal transform, shell sums, the logistic's
fixed point and limits."""
import numpy as np
import pytest
from numpy.polynomial import legendre as Lg

from oracle import indicator as IND
from workloads import states


def lt(i, s):
    e = np.zeros(i + 1)
    e[i] = 1.0
    return Lg.legval(s, e) * np.sqrt((2 * i + 1) / 2.0)


@pytest.mark.parametrize("N", [3, 4, 5])
def test_lgl_nodes_match_basis(oracle, N):
    assert np.abs(IND.lgl_nodes(N) - oracle.basis(N)[0]).max() < 1e-14


@pytest.mark.parametrize("N", [3, 4])
def test_single_mode_transform(N):
    xi = IND.lgl_nodes(N)
    X, Y = np.meshgrid(xi, xi)  # [b][a]
    for i in range(N + 1):
        for j in range(N + 1):
            q = lt(i, X) * lt(j, Y)
            m = IND.modal(q[None], N)[0]
            e = np.zeros((N + 1, N + 1))
            e[i, j] = 1.0
            assert np.abs(m - e).max() < 1e-12


def _state_from_rho_p(rho, p):
    return states.conservative(rho, 0.1 + 0 * rho, -0.2 + 0 * rho, p, 1.4)


@pytest.mark.parametrize("N", [3, 4])
def test_energy_closed_form(N):
    xi = IND.lgl_nodes(N)
    X, Y = np.meshgrid(xi, xi)
    c, a = 3.0, 0.05
    # rho p = c + a Lt_N(x): m_00 = 2c (Lt_0 Lt_0 = 1/2), m_N0 = a sqrt(2)
    rho = np.ones_like(X)[None]
    p = (c + a * lt(N, X))[None]
    E = IND.hennemann_energy(_state_from_rho_p(rho, p), N)[0]
    m00, mN0 = 2 * c, a * np.sqrt(2.0)
    assert abs(E - mN0 ** 2 / (m00 ** 2 + mN0 ** 2)) < 1e-14
    # second-highest mode is caught by the second fraction
    p2 = (c + a * lt(N - 1, Y))[None]
    E2 = IND.hennemann_energy(_state_from_rho_p(rho, p2), N)[0]
    assert abs(E2 - mN0 ** 2 / (m00 ** 2 + mN0 ** 2)) < 1e-14


@pytest.mark.parametrize("N", [3, 4])
def test_alpha_limits_and_fixed_point(N):
    T = IND.threshold(N)
    assert IND.hennemann_alpha_of_energy(np.array([0.0]), N)[0] == 0.0
    assert IND.hennemann_alpha_of_energy(np.array([1.0]), N)[0] == IND.ALPHA_MAX
    assert abs(IND.hennemann_alpha_of_energy(np.array([T]), N)[0] - 0.5) < 1e-15
    below = IND.hennemann_alpha_of_energy(np.array([0.9 * T]), N)[0]
    assert 0.0 <= below < 0.5
    es = np.linspace(0, 3 * T, 301)
    a = IND.hennemann_alpha_of_energy(es, N)
    assert (np.diff(a) >= 0).all()
    # a constant state has no modal energy above mode 0
    x = np.zeros((2, N + 1, N + 1))
    u = states.constant(x)
    assert (IND.hennemann(u, N) == 0.0).all()


@pytest.mark.parametrize("N", [3, 4])
def test_feature_shell_sums(N):
    x = np.random.default_rng(1).uniform(0, 1, (20, N + 1, N + 1))
    u = states.random_admissible(x, 4)
    f = IND.features(u, N)
    assert f.shape == (20, 16)
    assert (f >= 0).all() and (f <= 1 + 1e-15).all()
    rho, p = IND.prims(u)
    for k, q in enumerate((rho, p)):
        m2 = IND.modal(q, N) ** 2
        low = m2.sum(axis=-1)[:, :N - 3].sum(axis=1) / m2.sum(axis=(-2, -1))
        lowy = m2.sum(axis=-2)[:, :N - 3].sum(axis=1) / m2.sum(axis=(-2, -1))
        assert np.abs(f[:, 8 * k:8 * k + 4].sum(axis=1) + low - 1).max() < 1e-13
        assert np.abs(f[:, 8 * k + 4:8 * k + 8].sum(axis=1) + lowy - 1).max() < 1e-13


def test_feature_single_mode():
    N = 3
    xi = IND.lgl_nodes(N)
    X, Y = np.meshgrid(xi, xi)
    rho = (2.0 + 0 * X)[None]  # constant density: all energy in shell 0
    p = (1.0 + 0.3 * lt(2, X) * lt(1, Y))[None]
    f = IND.features(_state_from_rho_p(rho, p), N)[0]
    assert np.allclose(f[:8], [1, 0, 0, 0, 1, 0, 0, 0], atol=1e-14)
    m00, m21 = 2.0, 0.3
    tot = m00 ** 2 + m21 ** 2
    assert np.allclose(f[8:12], [m00 ** 2 / tot, 0, m21 ** 2 / tot, 0], atol=1e-14)
    assert np.allclose(f[12:16], [m00 ** 2 / tot, m21 ** 2 / tot, 0, 0], atol=1e-14)
