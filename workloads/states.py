"""Initial conditions of the synthetic workloads, evaluated at caller-supplied nodes.

Every function takes node coordinates x, y (arrays of shape [E, n, n], indexed
(e, b, a)) and returns the conservative state u with shape [E, 4, n, n],
variables (rho, rho v1, rho v2, rho e).
"""
import math

import numpy as np

from .rng import uniform


def conservative(rho, v1, v2, p, gamma):
    u = np.empty((rho.shape[0], 4) + rho.shape[1:])
    u[:, 0] = rho
    u[:, 1] = rho * v1
    u[:, 2] = rho * v2
    u[:, 3] = p / (gamma - 1.0) + 0.5 * rho * (v1 * v1 + v2 * v2)
    return u


def constant(x, rho=1.0, v1=0.3, v2=-0.2, p=1.0, gamma=1.4):
    one = np.ones_like(x)
    return conservative(rho * one, v1 * one, v2 * one, p * one, gamma)


def density_wave(x, y, gamma=1.4, t=0.0):
    """rho = 2 + 0.98 sin(2 pi (x + y - 0.3 t)), v = (0.1, 0.2), p = 20 (Sec. 3.1)."""
    rho = 2.0 + 0.98 * np.sin(2 * np.pi * (x + y - 0.3 * t))
    one = np.ones_like(x)
    return conservative(rho, 0.1 * one, 0.2 * one, 20.0 * one, gamma)


def isentropic_flow(x, y, gamma=3.0):
    """Cheng-Shu near-vacuum isentropic flow rotated by 45 degrees (Sec. 3.2), t = 0."""
    xp = (x + y) / math.sqrt(2.0)
    rho = 1.0 + 0.9999999 * np.sin(np.pi * xp)
    zero = np.zeros_like(x)
    return conservative(rho, zero, zero, rho ** gamma, gamma)


def vortex(x, y, seed=1, gamma=1.4, eps=5.0, R=0.1, xc=0.5, yc=0.5, amp=1e-3):
    """Isentropic vortex of strength eps on [0,1]^2 plus a seeded per-node density
    perturbation amp*(2U-1) at fixed velocity and pressure."""
    xb, yb = (x - xc) / R, (y - yc) / R
    r2 = xb * xb + yb * yb
    T = 1.0 - (gamma - 1.0) * eps * eps * np.exp(1.0 - r2) / (8.0 * gamma * np.pi * np.pi)
    rho = T ** (1.0 / (gamma - 1.0))
    s = eps / (2.0 * np.pi) * np.exp(0.5 * (1.0 - r2))
    v1, v2 = -s * yb, s * xb
    p = rho ** gamma
    k = np.arange(rho.size, dtype=np.uint64).reshape(rho.shape)
    rho = rho + amp * (2.0 * uniform(seed, k) - 1.0)
    return conservative(rho, v1, v2, p, gamma)


def sedov_gaussian(x, y, gamma=1.4, E0=1.0, sigma=0.06, p0=1e-5, xc=0.0, yc=0.0):
    """Blast: rho = 1, v = 0, p = p0 + (gamma-1) E0 exp(-r^2/(2 sigma^2)) / (2 pi sigma^2)."""
    r2 = (x - xc) ** 2 + (y - yc) ** 2
    p = p0 + (gamma - 1.0) * E0 * np.exp(-r2 / (2 * sigma * sigma)) / (2 * np.pi * sigma * sigma)
    one = np.ones_like(x)
    return conservative(one, 0 * one, 0 * one, p, gamma)


def sedov_tophat(x, y, gamma=1.4, e=1.0, r0=0.21875, p0=1e-5):
    """Blast with the energy in a disc of radius r0 (Sec. 3.4)."""
    r2 = x * x + y * y
    p = np.where(r2 <= r0 * r0, (gamma - 1.0) * e / (np.pi * r0 * r0), p0)
    one = np.ones_like(x)
    return conservative(one, 0 * one, 0 * one, p, gamma)


def shear_layer(x, y, seed=3, gamma=1.4, amp=0.1):
    """rho = 1 inside |y| < 0.5 else 0.5; v1 = +-0.5; v2 = amp sin(2 pi x + phi); p = 2.5."""
    phi = 2 * np.pi * float(uniform(seed, 0))
    inside = np.abs(y) < 0.5
    rho = np.where(inside, 1.0, 0.5)
    v1 = np.where(inside, 0.5, -0.5)
    v2 = amp * np.sin(2 * np.pi * x + phi)
    return conservative(rho, v1, v2, 2.5 * np.ones_like(x), gamma)


def quadrants(x, y, seed=5, gamma=1.4, xs=0.5, ys=0.5):
    """Four constant states on the quadrants of [0,1]^2 split at (xs, ys)."""
    q = (x >= xs).astype(np.int64) + 2 * (y >= ys).astype(np.int64)
    U = uniform(seed, np.arange(16, dtype=np.uint64)).reshape(4, 4)
    rho = 0.1 + 1.4 * U[:, 0]
    p = 0.03 + 1.47 * U[:, 1]
    v1 = -1.0 + 2.0 * U[:, 2]
    v2 = -1.0 + 2.0 * U[:, 3]
    return conservative(rho[q], v1[q], v2[q], p[q], gamma)


def random_admissible(shape_like, seed, gamma=1.4, rho_range=(0.2, 2.0), p_range=(0.1, 2.0),
                      vmax=1.0):
    """Independent random admissible states per node (for operator tests)."""
    n = shape_like.size
    k = np.arange(4 * n, dtype=np.uint64)
    U = uniform(seed, k).reshape(4, *shape_like.shape)
    rho = rho_range[0] + (rho_range[1] - rho_range[0]) * U[0]
    p = p_range[0] + (p_range[1] - p_range[0]) * U[1]
    v1 = vmax * (2 * U[2] - 1)
    v2 = vmax * (2 * U[3] - 1)
    return conservative(rho, v1, v2, p, gamma)


def workload_state(name, x, y, seed=None):
    """Initial state of the named workload at the given nodes."""
    if name == "vortex304":
        return vortex(x, y, seed=1 if seed is None else seed)
    if name == "blast22k":
        return sedov_gaussian(x, y)
    if name == "shear59k":
        return shear_layer(x, y, seed=3 if seed is None else seed)
    if name == "quadrants247k":
        return quadrants(x, y, seed=5 if seed is None else seed)
    raise ValueError(name)
