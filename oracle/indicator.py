"""Oracle for the modal troubled-cell indicator and the learned-indicator
features.  TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).  Plain numpy FP64.

Modal coefficients.  The nodal values q[b][a] of an element (a along x, b along
y, LGL nodes) interpolate q(x, y) = sum_ij m[i][j] Lt_i(x) Lt_j(y) with the
orthonormal Legendre polynomials Lt_i = sqrt((2i+1)/2) L_i on [-1, 1].  m is
the inverse of that interpolation, one direction at a time.

Hennemann indicator (Hennemann, Rueda-Ramirez, Hindenlang, Gassner 2021; the
paper uses it as its AMR indicator for shocks, Sec. 3.3 to 3.6, on q = rho p,
and, on q = p without the cap, as the weight of combined limiting, Sec. 3.5):
  E_all   = sum of m_ij^2 over all modes,
  E_low1  = sum over i, j <= N-1,   E_low2 = sum over i, j <= N-2,
  energy  = max((E_all - E_low1) / E_all, (E_low1 - E_low2) / E_low1),
  T       = 0.5 * 10^(-1.8 (N+1)^(1/4)),   s = ln((1 - 1e-4) / 1e-4),
  alpha   = 1 / (1 + exp(-(s / T) (energy - T))),
  alpha   = 0 below alpha_min = 1e-3, then capped at alpha_max = 0.5.

Features (16 per element, any N >= 3): for q in (rho, p), with E_q the sum of
all m_ij^2 of q, the x-shell fractions sum_j m_kj^2 / E_q and the y-shell
fractions sum_i m_ik^2 / E_q for the four highest shells k = N-3 .. N, in the
order [rho: x shells, rho: y shells, p: x shells, p: y shells].

Parity: the modal transform and the feature fractions are pinned by closed
forms (single modes, shell sums).  The indicator constants come from the cited
indicator paper, not from this paper; their values are "parity unpinned" here
beyond the logistic's fixed point alpha(T) = 1/2 and its limits.
"""
import numpy as np
from numpy.polynomial import legendre as Lg

ALPHA_MIN = 1e-3
ALPHA_MAX = 0.5


def lgl_nodes(N):
    """LGL nodes: the endpoints and the roots of P_N' (numpy Legendre series)."""
    c = np.zeros(N + 1)
    c[N] = 1.0
    inner = Lg.legroots(Lg.legder(c))
    return np.concatenate([[-1.0], np.sort(inner.real), [1.0]])


def vandermonde(N):
    """V[a][i] = Lt_i(xi_a), orthonormal Legendre at the LGL nodes."""
    xi = lgl_nodes(N)
    n = N + 1
    V = np.zeros((n, n))
    for i in range(n):
        e = np.zeros(n)
        e[i] = 1.0
        V[:, i] = Lg.legval(xi, e) * np.sqrt((2 * i + 1) / 2.0)
    return V


def modal(q, N):
    """q[..., b, a] nodal -> m[..., i, j] modal (i along x, j along y)."""
    Vi = np.linalg.inv(vandermonde(N))
    return np.einsum("ia,jb,...ba->...ij", Vi, Vi, q)


def prims(u, gamma=1.4):
    rho = u[:, 0]
    p = (gamma - 1.0) * (u[:, 3] - 0.5 * (u[:, 1] ** 2 + u[:, 2] ** 2) / rho)
    return rho, p


def hennemann_energy(u, N, gamma=1.4, quantity="rho_p"):
    rho, p = prims(u, gamma)
    m2 = modal(rho * p if quantity == "rho_p" else p, N) ** 2
    e_all = m2.sum(axis=(-2, -1))
    e_l1 = m2[..., :N, :N].sum(axis=(-2, -1))
    e_l2 = m2[..., :N - 1, :N - 1].sum(axis=(-2, -1))
    return np.maximum((e_all - e_l1) / e_all, (e_l1 - e_l2) / e_l1)


def threshold(N):
    return 0.5 * 10.0 ** (-1.8 * (N + 1) ** 0.25)


def hennemann_alpha_of_energy(energy, N, alpha_max=ALPHA_MAX):
    T = threshold(N)
    s = np.log((1.0 - 1e-4) / 1e-4)
    a = 1.0 / (1.0 + np.exp(-(s / T) * (energy - T)))
    a = np.where(a < ALPHA_MIN, 0.0, a)
    return np.minimum(a, alpha_max)


def hennemann(u, N, gamma=1.4):
    """Per-element indicator alpha in [0, alpha_max], FP64."""
    return hennemann_alpha_of_energy(hennemann_energy(u, N, gamma), N)


def shock_indicator(u, N, gamma=1.4):
    """The indicator of combined limiting (Sec. 3.5): the same logistic on the
    pressure's modal energy, not capped (alpha in [0, 1])."""
    return hennemann_alpha_of_energy(hennemann_energy(u, N, gamma, quantity="p"), N, alpha_max=1.0)


def features(u, N, gamma=1.4):
    """[E, 16] shell energy fractions of rho and p, FP64."""
    assert N >= 3
    rho, p = prims(u, gamma)
    out = []
    for q in (rho, p):
        m2 = modal(q, N) ** 2
        tot = m2.sum(axis=(-2, -1))[:, None]
        xs = m2.sum(axis=-1)[:, N - 3:] / tot  # x-mode shells k: sum over j of m[k][j]^2
        ys = m2.sum(axis=-2)[:, N - 3:] / tot
        out += [xs, ys]
    return np.concatenate(out, axis=1)
