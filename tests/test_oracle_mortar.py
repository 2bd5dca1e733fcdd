"""Pins of the oracle's mortar limiter (Sec. 2.3, Mortar Limiting) at fractional
factors, positivity mode (eq. Bounds_Positivity, eq. BlendingFluxes_alpha).

The oracle limits the high-order mortar correction with one factor theta_S per
mortar: the largest theta in [0, 1] for which every node i of the mortar stays
within its bounds when it takes n_i times its share theta c^S_i, where n_i is
the number of mortars that contain the node (the remark on mortar limiting
scales by n_i so that the corrections of all mortars at a node can be taken
together).  The bounds are rho >= beta rho^FV and p >= beta p(u^FV), and the
base state is u^vol, the state after the volume limiter.

These tests recompute theta_S by brute force from quantities that do not go
through the oracle's factor code: u^FV from the oracle's low-order residual,
n_i by counting mortar slots in the mesh's mortar table, the node of each slot
from the face geometry, and the factor itself by scanning theta on a grid
(coarse, then refined around the first infeasible point: the feasible set of
each node is an interval containing 0, since rho is linear and p concave along
the ray).  The states are chosen so that the factors are strictly between 0
and 1, and some mortars contain nodes on two mortars (n_i = 2).
"""
import numpy as np
import pytest

import oracle as O
from workloads import states
from workloads.meshes import build, refined_box_mesh, workload_mesh
from workloads.rng import uniform

GAMMA = 1.4


def pressure(q):
    return (GAMMA - 1.0) * (q[..., 3] - 0.5 * (q[..., 1] ** 2 + q[..., 2] ** 2) / q[..., 0])


def slot_nodes(M):
    """(element, a, b) of every mortar slot, [M, 3n, 3]: the large face's n
    nodes, then each small face's n nodes, each by position along its face."""
    N, n = M.N, M.n
    out = np.zeros((M.M, 3 * n, 3), dtype=np.int64)
    for S, (large, face, s0, s1) in enumerate(M.mortars()):
        for s in range(3 * n):
            e, f = (large, face) if s < n else ((s0, face ^ 1) if s < 2 * n else (s1, face ^ 1))
            k = s % n
            a, b = {0: (0, k), 1: (N, k), 2: (k, 0), 3: (k, N)}[f]
            out[S, s] = (e, a, b)
    return out


def mortar_counts(nodes):
    """n_i for every slot: how many slots of all mortars sit on its node."""
    keys = [tuple(x) for x in nodes.reshape(-1, 3)]
    cnt = {}
    for k in keys:
        cnt[k] = cnt.get(k, 0) + 1
    return np.array([cnt[k] for k in keys]).reshape(nodes.shape[:2])


def feasible(uvol, dc, rmin, pmin, th):
    """all nodes (rows) of the mortar within bounds at factor th"""
    q = uvol + th * dc
    return bool(np.all(q[:, 0] >= rmin) and np.all(q[:, 0] > 0) and np.all(pressure(q) >= pmin))


def brute_theta(uvol, dc, rmin, pmin, h=1e-6):
    """largest grid point theta in [0, 1] (grid h) keeping every node within bounds"""
    if not feasible(uvol, dc, rmin, pmin, 0.0):
        return 0.0
    if feasible(uvol, dc, rmin, pmin, 1.0):
        return 1.0
    lo, step = 0.0, 1e-3
    while step >= h * 0.999:
        t = lo
        while t + step <= 1.0 and feasible(uvol, dc, rmin, pmin, t + step):
            t += step
        lo = t
        step *= 1e-1
    return lo


def run_case(N, spec, u, cfl, beta):
    M = O.Mesh(N, *spec.args())
    dt = M.max_dt(u, cfl)
    out, st, uvol, dslot, theta = M.fe_step_detail(u, dt, beta=beta)
    assert st["violations"] == 0 and st["fv_inadmissible"] == 0
    _, _, m = M.geometry()
    ufv = u + dt * M.rhs(u, O.RHS_LOW)
    rmin = beta * ufv[:, 0]                                   # [E, n, n] (b, a)
    pmin = beta * pressure(np.moveaxis(ufv, 1, -1))
    nodes = slot_nodes(M)
    ni = mortar_counts(nodes)
    return M, dt, out, uvol, dslot, theta, m, rmin, pmin, nodes, ni


def mortar_rays(S, dt, uvol, dslot, m, rmin, pmin, nodes, ni, scale_by_ni=True):
    e, a, b = nodes[S, :, 0], nodes[S, :, 1], nodes[S, :, 2]
    c = dt / m[e, b, a][:, None] * dslot[S]
    k = ni[S][:, None] if scale_by_ni else 1.0
    return uvol[e, :, b, a], k * c, rmin[e, b, a], pmin[e, b, a]


def smooth_cases():
    """states on the 304-leaf mesh (16 mortars, corner nodes on two mortars)
    for which every mortar factor of the strict bounds beta = 0.999 lies
    strictly between 0 and 1"""
    spec = workload_mesh("vortex304")
    out = []
    for N in (3, 4):
        x, y, _ = O.Mesh(N, *spec.args()).geometry()
        r = np.hypot(x - 0.5, y - 0.5)
        tanh = np.tanh((r - 0.12) / 0.02)
        out.append((N, spec, states.vortex(x, y, seed=1, amp=0.0), 0.9, 0.999))
        out.append((N, spec, states.conservative(1 + 0.95 * tanh, 0 * x, 0 * x, 0.05 + (1 - tanh), GAMMA),
                    0.9, 0.999))
    return out


def blast_case(N, seed):
    """a circular jump of density and pressure on an 8^2 mesh whose central
    4^2 cells are refined once (16 mortars); with the paper's beta = 0.1 a
    few seeds give fractional mortar factors"""
    spec = refined_box_mesh(8, (0.25, 0.25), (0.75, 0.75), 0.0, 0.0, 1.0)
    x, y, _ = O.Mesh(N, *spec.args()).geometry()
    r = uniform(seed, np.arange(8, dtype=np.uint64))
    inside = (x - (0.25 + 0.5 * r[0])) ** 2 + (y - (0.25 + 0.5 * r[1])) ** 2 < (0.05 + 0.3 * r[2]) ** 2
    rho = np.where(inside, 10 ** (-3 * r[3]), 10 ** (-3 * r[4]))
    p = np.where(inside, 10 ** (2 - 5 * r[5]), 10 ** (2 - 5 * r[6]))
    vx = (r[7] - 0.5) * 4 * np.ones_like(x)
    return N, spec, states.conservative(rho, vx, 0 * vx, p, GAMMA), 1.0, 0.1


def l_mesh():
    """8^2 periodic mesh whose cells in an L-shaped region are refined once:
    the coarse cell in the notch of the L has mortars on two adjacent faces,
    so its corner node is on two mortars (n_i = 2) with a nonzero correction
    (at the outer end of a small face the interpolated state is the large
    face's end state, the high- and low-order mortar fluxes coincide there and
    a small-side corner contributes nothing)"""
    def pred(x, y, l):
        return (0.5 < x < 0.75 and 0.25 < y < 0.75) or (0.25 < x < 0.5 and 0.5 < y < 0.75)
    return build((0.0, 0.0, 1.0, 1.0, 8, 8), pred, 1)


def l_cases():
    spec = l_mesh()
    out = []
    for N, kind, beta in ((4, "vortex", 0.999), (4, "wave", 0.99), (3, "wave", 0.999)):
        x, y, _ = O.Mesh(N, *spec.args()).geometry()
        if kind == "vortex":
            u = states.vortex(x, y, seed=1, amp=0.0)
        else:
            u = states.conservative(1 + 0.5 * np.sin(2 * np.pi * (x + 2 * y)), 0.3 + 0 * x, -0.2 + 0 * x,
                                    1 + 0.5 * np.cos(2 * np.pi * (3 * x - y)), GAMMA)
        out.append((N, spec, u, 0.9, beta))
    return out


CASES = smooth_cases() + [blast_case(3, 77), blast_case(4, 589)] + l_cases()
IDS = ["vortex-N3", "tanh-N3", "vortex-N4", "tanh-N4", "blast77-N3-beta0.1", "blast589-N4-beta0.1",
       "L-vortex-N4", "L-wave-N4", "L-wave-N3"]


@pytest.mark.parametrize("case", range(len(CASES)), ids=IDS)
def test_mortar_factor_equals_brute_force(case):
    N, spec, u, cfl, beta = CASES[case]
    M, dt, out, uvol, dslot, theta, m, rmin, pmin, nodes, ni = run_case(N, spec, u, cfl, beta)
    frac = np.nonzero((theta > 0) & (theta < 1))[0]
    assert len(frac) >= 1
    for S in range(M.M):
        q, dc, rm, pm = mortar_rays(S, dt, uvol, dslot, m, rmin, pmin, nodes, ni)
        tb = brute_theta(q, dc, rm, pm)
        # the oracle aims at bounds raised by 2^-41: it may lie below the
        # brute-force grid point by that much, and above it by one grid step
        assert tb - 1e-9 <= theta[S] <= tb + 1e-6 + 1e-12, (S, theta[S], tb)


@pytest.mark.parametrize("case", range(len(CASES)), ids=IDS)
def test_mortar_correction_is_applied_once_per_mortar(case):
    """u_new = u_vol + sum over the node's mortars (ascending id) of
    theta_S c^S_i: the correction itself is not scaled by n_i"""
    N, spec, u, cfl, beta = CASES[case]
    M, dt, out, uvol, dslot, theta, m, rmin, pmin, nodes, ni = run_case(N, spec, u, cfl, beta)
    ref = uvol.copy()
    for S in range(M.M):
        if theta[S] == 0.0:  # (an undefined high-order mortar flux is not applied)
            continue
        for s in range(3 * M.n):
            e, a, b = nodes[S, s]
            ref[e, :, b, a] += theta[S] * dt / m[e, b, a] * dslot[S, s]
    scale = np.abs(ref).max(axis=(0, 2, 3))[None, :, None, None]
    assert np.max(np.abs(out - ref) / scale) < 1e-14


def test_fractional_factors_cover_two_mortar_nodes_and_depend_on_n_i():
    """On the L-shaped refinement: fractional mortars contain large-side nodes
    with n_i = 2 and a nonzero correction, and the brute force with n_i = 1
    everywhere gives a different factor for some of them, so a dropped or
    wrong n_i would fail the pin above."""
    two, differs = 0, 0
    for N, spec, u, cfl, beta in CASES[6:]:
        M, dt, out, uvol, dslot, theta, m, rmin, pmin, nodes, ni = run_case(N, spec, u, cfl, beta)
        for S in range(M.M):
            if not 0.0 < theta[S] < 1.0:
                continue
            if np.any((ni[S] == 2) & np.any(dslot[S] != 0.0, axis=1)):
                two += 1
            q, dc, rm, pm = mortar_rays(S, dt, uvol, dslot, m, rmin, pmin, nodes, ni, scale_by_ni=False)
            if abs(brute_theta(q, dc, rm, pm, h=1e-4) - theta[S]) > 1e-3:
                differs += 1
    assert two >= 2
    assert differs >= 2


def test_mortar_factors_are_strictly_fractional_under_strict_bounds():
    """the cases above do exercise the fractional branch: all 16 mortar
    factors of the N = 3 strict-bound vortex are in (0, 1)"""
    N, spec, u, cfl, beta = CASES[0]
    theta = run_case(N, spec, u, cfl, beta)[5]
    assert np.all((theta > 0) & (theta < 1))
