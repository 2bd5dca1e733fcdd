"""Parity metrics between the GPU library and the oracle (tolerance 1e-12).

States: |g - c| <= tol * s per DOF, with the scale
  s = max(|c_v|, 1e-3 max|c_v|, q_v),  q_rho = rho, q_m = rho c, q_E = E
of the oracle's node state (c = sound speed).  A momentum cannot be resolved
better than the pressure terms that change it, whose size is rho c per unit
Courant number; without that floor a momentum that starts at zero would be
compared at the level of its own round-off.
Time derivatives: |g - c| <= tol * T_v per variable, T_v the largest single
flux-difference term (|f_v| + lambda |u_v|) / (h w_0 / 2) of the state (w_0 the
smallest LGL weight, lambda = |v_n| + c): the residual is a sum of such terms
with cancellations.
Both sides agree on where the scheme is undefined (NaN); those entries are
required to be NaN on both sides and are otherwise excluded.
"""
import numpy as np


def _prims(u, gamma):
    rho = u[:, 0]
    v1, v2 = u[:, 1] / rho, u[:, 2] / rho
    p = (gamma - 1) * (u[:, 3] - 0.5 * rho * (v1 * v1 + v2 * v2))
    c = np.sqrt(np.abs(gamma * p / rho))
    return rho, v1, v2, p, c


def state_err(g, c, gamma=1.4):
    """Worst scaled error per the state metric."""
    g, c = np.asarray(g), np.asarray(c)
    rho, v1, v2, p, cs = _prims(c, gamma)
    q = np.stack([np.abs(rho), np.abs(rho) * cs, np.abs(rho) * cs, np.abs(c[:, 3])], axis=1)
    floor = 1e-3 * np.abs(c).max(axis=(0, 2, 3), keepdims=True)
    den = np.maximum(np.maximum(np.abs(c), floor), q)
    return float((np.abs(g - c) / den).max())


def rate_err(g, c, u, x, y, w0, gamma=1.4):
    """Worst error of du/dt relative to the flux-term scale; NaN must match."""
    g, c = np.asarray(g), np.asarray(c)
    ng, nc = ~np.isfinite(g), ~np.isfinite(c)
    assert np.array_equal(ng, nc), "the two sides disagree on where the scheme is undefined"
    rho, v1, v2, p, cs = _prims(u, gamma)
    hx = (x[:, 0, -1] - x[:, 0, 0])[:, None, None]
    hy = (y[:, -1, 0] - y[:, 0, 0])[:, None, None]
    fx = np.stack([rho * v1, rho * v1 * v1 + p, rho * v1 * v2, (u[:, 3] + p) * v1], axis=1)
    fy = np.stack([rho * v2, rho * v1 * v2, rho * v2 * v2 + p, (u[:, 3] + p) * v2], axis=1)
    # flux terms plus the LLF dissipation terms lambda |u|
    lx = (np.abs(v1) + cs)[:, None] * np.abs(u)
    ly = (np.abs(v2) + cs)[:, None] * np.abs(u)
    T = ((np.abs(fx) + lx) / hx[:, None] + (np.abs(fy) + ly) / hy[:, None]) * 2.0 / w0
    T = T.max(axis=(0, 2, 3), keepdims=True)
    d = np.where(nc, 0.0, np.abs(g - c))
    return float((d / T).max())
