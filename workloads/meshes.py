"""Quadtree leaf lists for the synthetic workloads.

A mesh is a periodic box [x0, x0+Lx] x [y0, y0+Ly] with an nx0 x ny0 root grid;
a leaf (level, ix, iy) covers cell (ix, iy) of the (nx0 2^level) x (ny0 2^level)
grid.  Leaves are refined by a predicate on their centre and then 2:1 balanced
across faces (periodic).  Output order is Morton (Z) order of the leaves.
"""
from dataclasses import dataclass

import numpy as np


@dataclass
class MeshSpec:
    level: np.ndarray
    ix: np.ndarray
    iy: np.ndarray
    x0: float
    y0: float
    Lx: float
    Ly: float
    nx0: int
    ny0: int

    @property
    def E(self):
        return len(self.level)

    def args(self):
        return (self.level, self.ix, self.iy, self.x0, self.y0, self.Lx, self.Ly, self.nx0, self.ny0)

    def counts(self):
        lv, c = np.unique(self.level, return_counts=True)
        return dict(zip(lv.tolist(), c.tolist()))


def _centre(box, l, i, j):
    x0, y0, Lx, Ly, nx0, ny0 = box
    hx, hy = Lx / (nx0 << l), Ly / (ny0 << l)
    return x0 + (i + 0.5) * hx, y0 + (j + 0.5) * hy


def _balance(leaves, nx0, ny0):
    """Refine leaves until neighbours across faces differ by at most one level."""
    changed = True
    while changed:
        changed = False
        to_split = set()
        for (l, i, j) in leaves:
            if l < 2:
                continue
            nxl, nyl = nx0 << l, ny0 << l
            for di, dj in ((1, 0), (-1, 0), (0, 1), (0, -1)):
                ci, cj = (i + di) % nxl, (j + dj) % nyl
                # the leaf containing the neighbour cell, searched at coarser levels
                for lc in range(l - 2, -1, -1):
                    s = l - lc
                    key = (lc, ci >> s, cj >> s)
                    if key in leaves:
                        to_split.add(key)
                        break
        if to_split:
            changed = True
            for key in to_split:
                leaves.discard(key)
                l, i, j = key
                for a in (0, 1):
                    for b in (0, 1):
                        leaves.add((l + 1, 2 * i + a, 2 * j + b))
    return leaves


def _morton(l, i, j, L):
    s = L - l
    x, y = i << s, j << s
    key = 0
    for bit in range(max(L, 1) + 12):
        key |= ((x >> bit) & 1) << (2 * bit)
        key |= ((y >> bit) & 1) << (2 * bit + 1)
    return key


def build(box, predicate, maxlev):
    """Refine every leaf of level < maxlev whose centre satisfies predicate(x, y, level)."""
    x0, y0, Lx, Ly, nx0, ny0 = box
    leaves = {(0, i, j) for i in range(nx0) for j in range(ny0)}
    for lev in range(maxlev):
        split = [k for k in leaves if k[0] == lev and predicate(*_centre(box, *k), lev)]
        for key in split:
            leaves.discard(key)
            l, i, j = key
            for a in (0, 1):
                for b in (0, 1):
                    leaves.add((l + 1, 2 * i + a, 2 * j + b))
        _balance(leaves, nx0, ny0)
    return to_spec(box, leaves)


def to_spec(box, leaves):
    x0, y0, Lx, Ly, nx0, ny0 = box
    L = max(l for l, _, _ in leaves)
    order = sorted(leaves, key=lambda k: _morton(*k, L))
    arr = np.array(order, dtype=np.int64).reshape(-1, 3)
    return MeshSpec(arr[:, 0].astype(np.int8), arr[:, 1].astype(np.int32),
                    arr[:, 2].astype(np.int32), x0, y0, Lx, Ly, nx0, ny0)


def uniform_mesh(nx0, ny0, x0=0.0, y0=0.0, Lx=1.0, Ly=1.0):
    return build((x0, y0, Lx, Ly, nx0, ny0), lambda x, y, l: False, 0)


def refined_box_mesh(n_base, box_lo, box_hi, x0, y0, L):
    """n_base^2 square elements on [x0,x0+L]^2, elements with centre inside the box refined once."""
    (bx0, by0), (bx1, by1) = box_lo, box_hi
    return build((x0, y0, L, L, n_base, n_base),
                 lambda x, y, l: bx0 < x < bx1 and by0 < y < by1, 1)


WORKLOADS = ("vortex304", "blast22k", "shear59k", "quadrants247k")


def workload_mesh(name):
    """Leaf lists of the named synthetic workloads (name = initial state + leaf count)."""
    if name == "vortex304":  # [0,1]^2, 16^2 base, +1 level in [0.375, 0.625]^2
        return refined_box_mesh(16, (0.375, 0.375), (0.625, 0.625), 0.0, 0.0, 1.0)
    if name == "blast22k":  # blast on [-1,1]^2, 64^2 base, +3 levels where r <= 0.3
        return build((-1.0, -1.0, 2.0, 2.0, 64, 64), lambda x, y, l: x * x + y * y <= 0.09, 3)
    if name == "shear59k":  # [-1,1]^2, 128^2 base, +3 levels on leaves meeting |(|y| - 0.5)| < 0.0175
        return build((-1.0, -1.0, 2.0, 2.0, 128, 128),
                     lambda x, y, l: abs(abs(y) - 0.5) < 0.0175 + 0.5 * 2.0 / (128 << l), 3)
    if name == "quadrants247k":  # four quadrants on [0,1]^2, 256^2 base, +2 levels near x, y in {0, 0.5}

        def near(x, y, l):  # leaf meets the band of half-width 0.022 around a line
            def d(t):
                return min(abs(t), abs(t - 0.5), abs(t - 1.0))
            return min(d(x), d(y)) < 0.022 + 0.5 / (256 << l)

        return build((0.0, 0.0, 1.0, 1.0, 256, 256), near, 2)
    raise ValueError(name)


def workload_order(name):
    """Polynomial degree N of a named workload."""
    return 4 if name == "quadrants247k" else 3


def random_mesh(seed, n_base=4, maxlev=2, frac=0.35, L=1.0, x0=0.0, y0=0.0):
    """Seeded random 2:1-balanced refinement of an n_base^2 periodic grid."""
    from .rng import uniform

    box = (x0, y0, L, L, n_base, n_base)
    leaves = {(0, i, j) for i in range(n_base) for j in range(n_base)}
    for lev in range(maxlev):
        cand = sorted(k for k in leaves if k[0] == lev)
        u = uniform(seed * 1000 + lev, np.arange(len(cand), dtype=np.uint64))
        for key, r in zip(cand, u):
            if r < frac:
                leaves.discard(key)
                l, i, j = key
                for a in (0, 1):
                    for b in (0, 1):
                        leaves.add((l + 1, 2 * i + a, 2 * j + b))
        _balance(leaves, n_base, n_base)
    return to_spec(box, leaves)


def random_flags(spec, seed, p_refine=0.15, p_coarsen=0.5):
    """Seeded refine (+1) / coarsen (-1) / keep (0) flags for the leaves of spec.
    A leaf is flagged +1 with probability p_refine; the leaves of a parent cell
    are flagged -1 together with probability p_coarsen (so that whole sibling
    groups ask to be coarsened), unless flagged +1."""
    from .rng import uniform

    E = spec.E
    lev = spec.level.astype(np.int64)
    ur = uniform(seed, np.arange(E, dtype=np.uint64))
    # one draw per parent cell, keyed by (level, parent ix, parent iy)
    pkey = (lev << 50) | ((spec.ix.astype(np.int64) >> 1) << 25) | (spec.iy.astype(np.int64) >> 1)
    uc = uniform(seed + 7919, pkey.astype(np.uint64))
    flags = np.zeros(E, dtype=np.int8)
    flags[(uc < p_coarsen) & (lev > 0)] = -1
    flags[ur < p_refine] = 1
    return flags
