"""Pins of the oracle's one-dimensional operators against the paper and against
independent constructions (numpy's Legendre module)."""
import numpy as np
import pytest
from numpy.polynomial import legendre as npleg

from paper_values import exact, tables

T = tables()


@pytest.mark.parametrize("N", [3, 4, 5])
def test_lgl_weights_match_paper(oracle, N):
    """App. A prints the LGL weights for N = 3, 4, 5."""
    xi, w, D, S = oracle.basis(N)
    ref = np.array([exact(s) for s in T["lgl_weights"][str(N)]])
    assert np.max(np.abs(w - ref)) < 1e-15
    assert abs(w.sum() - 2.0) < 1e-15


@pytest.mark.parametrize("N", [1, 2, 3, 4, 5, 6, 7])
def test_lgl_nodes_are_lobatto(oracle, N):
    """Interior nodes are the roots of P_N' (numpy), endpoints are -1, 1."""
    xi, w, D, S = oracle.basis(N)
    c = np.zeros(N + 1)
    c[N] = 1.0
    roots = np.sort(npleg.legroots(npleg.legder(c))) if N > 1 else np.array([])
    assert np.allclose(xi[1:-1], roots, atol=1e-14, rtol=0)
    assert xi[0] == -1.0 and xi[-1] == 1.0


@pytest.mark.parametrize("N", [2, 3, 4, 5, 7])
def test_sbp_operators(oracle, N):
    """Qbar + Qbar^T = Bbar (summation by parts), Sbar = 2 Qbar - Bbar skew-symmetric,
    D differentiates polynomials of degree <= N exactly (Sec. 2.1)."""
    xi, w, D, S = oracle.basis(N)
    Q = np.diag(w) @ D
    B = np.zeros((N + 1, N + 1))
    B[0, 0], B[N, N] = -1.0, 1.0
    assert np.max(np.abs(Q + Q.T - B)) < 1e-13
    assert np.max(np.abs(S + S.T)) < 1e-13
    assert np.max(np.abs(S - (2 * Q - B))) < 1e-13
    # row sums of Sbar = -Bbar_aa, so telescoped subcell fluxes of a constant state equal f
    assert np.allclose(S.sum(axis=1), -np.diag(B), atol=1e-13)
    rng = np.random.default_rng(0)
    c = rng.standard_normal(N + 1)
    f = npleg.legval(xi, c)
    df = npleg.legval(xi, npleg.legder(c))
    assert np.max(np.abs(D @ f - df)) < 1e-11 * (1 + np.abs(df).max())


@pytest.mark.parametrize("N", [3, 4, 5])
def test_sparse_weights_match_paper_tables(oracle, N):
    """App. A, Tables local_weights and local_weights_4_5 (exact values)."""
    I, P, W = oracle.mortar_ops(N)
    ref = np.array([[exact(s) for s in row] for row in T["sparse_weights"][str(N)]])
    assert ref.shape == W.shape
    assert np.max(np.abs(W - ref)) < 5e-16
    assert np.array_equal(W > 0, ref > 0)  # sparsity pattern identical


@pytest.mark.parametrize("N", [1, 2, 3, 4, 5, 6, 7])
def test_sparse_weight_sums(oracle, N):
    """eq. sum_local_omega: row sums = large-face weights, column sums = small-face weights."""
    xi, w, D, S = oracle.basis(N)
    I, P, W = oracle.mortar_ops(N)
    assert np.allclose(W.sum(axis=1), w, atol=1e-14)
    assert np.allclose(W.sum(axis=0), np.concatenate([w, w]) / 2, atol=1e-14)
    assert (W >= 0).all()


@pytest.mark.parametrize("N", [1, 2, 3, 4, 5, 6, 7])
def test_sparse_weights_reduce_to_conforming(oracle, N):
    """eq. mortarfluxforconforminginterface: on matching faces the weights are
    delta_ij omega_i, so the mortar flux is the conforming flux."""
    xi, w, D, S = oracle.basis(N)
    W = oracle.overlap_weights(N, 1.0, 0.0)
    assert np.allclose(W, np.diag(w), atol=1e-15, rtol=0)


@pytest.mark.parametrize("N", [1, 3, 4, 6])
def test_interpolation_and_projection(oracle, N):
    """Mortar interpolation is exact on degree-N polynomials; the L2 projection of a
    per-half polynomial is the least-squares fit computed independently by
    Gauss-Legendre quadrature in numpy; projection conserves the integral."""
    xi, w, D, S = oracle.basis(N)
    I, P, W = oracle.mortar_ops(N)
    rng = np.random.default_rng(1)
    c = rng.standard_normal(N + 1)
    f = npleg.legval(xi, c)
    for h, sh in ((0, -1.0), (1, 1.0)):
        assert np.max(np.abs(I[h] @ f - npleg.legval((xi + sh) / 2, c))) < 1e-13
    # projection of a global polynomial restricted to the halves reproduces it
    g = [I[0] @ f, I[1] @ f]
    assert np.max(np.abs(P[0] @ g[0] + P[1] @ g[1] - f)) < 1e-13
    # independent L2 projection of a discontinuous per-half polynomial
    g0, g1 = rng.standard_normal(N + 1), rng.standard_normal(N + 1)
    gx, gw = npleg.leggauss(2 * N + 4)
    # Lagrange interpolants through the LGL nodes, evaluated in numpy
    def lag(vals, s):
        V = np.vander(xi, N + 1, increasing=True)
        coef = np.linalg.solve(V, vals)
        return np.polyval(coef[::-1], s)
    coeffs = []
    for m in range(N + 1):
        em = np.zeros(m + 1)
        em[m] = 1
        integ = 0.5 * np.sum(gw * lag(g0, gx) * npleg.legval((gx - 1) / 2, em))
        integ += 0.5 * np.sum(gw * lag(g1, gx) * npleg.legval((gx + 1) / 2, em))
        coeffs.append((2 * m + 1) / 2 * integ)
    ref = npleg.legval(xi, np.array(coeffs))
    assert np.max(np.abs(P[0] @ g0 + P[1] @ g1 - ref)) < 1e-13
    # conservation: sum_k w_k (Pg)_k = 1/2 sum_h sum_l w_l g^h_l
    lhs = w @ (P[0] @ g0 + P[1] @ g1)
    rhs = 0.5 * (w @ g0 + w @ g1)
    assert abs(lhs - rhs) < 1e-14
