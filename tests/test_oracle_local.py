"""Pins of the oracle's local limiting (eq. Bounds_Barstates): the bar state against
the exact Riemann solution, the bounds against the low-order graph, the low-order
state against its bounds, the entropy root against bisection, and the limited
scheme against the paper's convergence table with local limiting."""
import numpy as np
import pytest

from paper_values import tables
from test_oracle_scheme import _edges, _l2_errors, make
from workloads import states
from workloads.meshes import random_mesh, refined_box_mesh

T = tables()
G = 1.4


def _cons(rho, v1, v2, p):
    return states.conservative(*[np.array([x], dtype=float) for x in (rho, v1, v2, p)], G)[0]


# ---------------------------------------------------------------------------
# exact Riemann solver of the 1D Euler equations (Toro, Riemann Solvers and
# Numerical Methods for Fluid Dynamics, ch. 4), with a passive tangential velocity
# ---------------------------------------------------------------------------
def _fK(p, rK, pK, g):
    cK = np.sqrt(g * pK / rK)
    if p > pK:
        A, B = 2.0 / ((g + 1) * rK), (g - 1) / (g + 1) * pK
        f = (p - pK) * np.sqrt(A / (p + B))
        df = np.sqrt(A / (p + B)) * (1 - (p - pK) / (2 * (B + p)))
    else:
        f = 2 * cK / (g - 1) * ((p / pK) ** ((g - 1) / (2 * g)) - 1)
        df = 1.0 / (rK * cK) * (p / pK) ** (-(g + 1) / (2 * g))
    return f, df


def _star(WL, WR, g):
    (rL, uL, pL), (rR, uR, pR) = WL, WR
    p = 0.5 * (pL + pR)
    for _ in range(100):
        fL, dL = _fK(p, rL, pL, g)
        fR, dR = _fK(p, rR, pR, g)
        pn = max(p - (fL + fR + uR - uL) / (dL + dR), 1e-14)
        if abs(pn - p) < 1e-15 * p:
            p = pn
            break
        p = pn
    fL, _ = _fK(p, rL, pL, g)
    fR, _ = _fK(p, rR, pR, g)
    return p, 0.5 * (uL + uR) + 0.5 * (fR - fL)


def _riemann_pieces(WL, WR, g):
    """Breakpoints (wave speeds) and the sampler w(xi) = (rho, u, p, side)."""
    (rL, uL, pL), (rR, uR, pR) = WL, WR
    cL, cR = np.sqrt(g * pL / rL), np.sqrt(g * pR / rR)
    ps, us = _star(WL, WR, g)
    gm = (g - 1) / (g + 1)
    if ps > pL:
        rsL = rL * (ps / pL + gm) / (gm * ps / pL + 1)
        SL = uL - cL * np.sqrt((g + 1) / (2 * g) * ps / pL + (g - 1) / (2 * g))
        left = [SL]
    else:
        rsL = rL * (ps / pL) ** (1 / g)
        left = [uL - cL, us - cL * (ps / pL) ** ((g - 1) / (2 * g))]
    if ps > pR:
        rsR = rR * (ps / pR + gm) / (gm * ps / pR + 1)
        SR = uR + cR * np.sqrt((g + 1) / (2 * g) * ps / pR + (g - 1) / (2 * g))
        right = [SR]
    else:
        rsR = rR * (ps / pR) ** (1 / g)
        right = [us + cR * (ps / pR) ** ((g - 1) / (2 * g)), uR + cR]

    def w(xi):
        if xi < us:  # left of the contact
            if len(left) == 1:
                return (rL, uL, pL, 0) if xi < left[0] else (rsL, us, ps, 0)
            if xi < left[0]:
                return (rL, uL, pL, 0)
            if xi > left[1]:
                return (rsL, us, ps, 0)
            t = 2 / (g + 1) + (g - 1) / ((g + 1) * cL) * (uL - xi)
            return (rL * t ** (2 / (g - 1)), 2 / (g + 1) * (cL + (g - 1) / 2 * uL + xi),
                    pL * t ** (2 * g / (g - 1)), 0)
        if len(right) == 1:
            return (rR, uR, pR, 1) if xi > right[0] else (rsR, us, ps, 1)
        if xi > right[1]:
            return (rR, uR, pR, 1)
        if xi < right[0]:
            return (rsR, us, ps, 1)
        t = 2 / (g + 1) - (g - 1) / ((g + 1) * cR) * (uR - xi)
        return (rR * t ** (2 / (g - 1)), 2 / (g + 1) * (-cR + (g - 1) / 2 * uR + xi),
                pR * t ** (2 * g / (g - 1)), 1)

    return sorted(left + [us] + right), w


def _fan_average(uL, uR, d, lam, g):
    """Mean of the exact Riemann solution of uL | uR along direction d over
    x / t in [-lam, lam] (conserved variables), by Gauss-Legendre quadrature on
    each smooth piece; returns also the extreme wave speed."""
    t_ = 1 - d  # tangential index

    def prim(u):
        r = u[0]
        return r, u[1 + d] / r, u[1 + t_] / r, (g - 1) * (u[3] - 0.5 * (u[1] ** 2 + u[2] ** 2) / r)

    rL, vnL, vtL, pL = prim(uL)
    rR, vnR, vtR, pR = prim(uR)
    brk, w = _riemann_pieces((rL, vnL, pL), (rR, vnR, pR), g)
    xs, ws = np.polynomial.legendre.leggauss(40)
    edges = [-lam] + [b for b in brk if -lam < b < lam] + [lam]
    acc = np.zeros(4)
    for a, b in zip(edges[:-1], edges[1:]):
        for x, wq in zip(xs, ws):
            xi = 0.5 * (a + b) + 0.5 * (b - a) * x
            r, vn, p, side = w(xi)
            vt = vtL if side == 0 else vtR
            q = np.zeros(4)
            q[0], q[1 + d], q[1 + t_] = r, r * vn, r * vt
            q[3] = p / (g - 1) + 0.5 * r * (vn * vn + vt * vt)
            acc += 0.5 * (b - a) * wq * q
    return acc / (2 * lam), max(abs(brk[0]), abs(brk[-1]))


RIEMANN = [
    # (rho, v1, v2, p) left and right
    ((1.0, 0.3, -0.2, 1.0), (0.7, -0.1, 0.4, 0.6)),    # shock and rarefaction
    ((1.2, -0.5, 0.1, 0.4), (1.0, 0.6, 0.0, 0.5)),     # two rarefactions
    ((0.8, 0.9, 0.3, 1.5), (1.1, -0.4, -0.3, 1.2)),    # two shocks
    ((1.0, 0.2, 0.5, 1.0), (0.4, 0.2, -0.5, 1.0)),     # contact and shear only
]


@pytest.mark.parametrize("case", range(len(RIEMANN)))
@pytest.mark.parametrize("d", [0, 1])
def test_bar_state_is_riemann_fan_average(oracle, case, d):
    """The bar state is the mean of the exact Riemann solution over the fan
    [-lambda t, lambda t] (the integral form of the conservation law over that box;
    Sec. 2.2 interprets it as the intermediate state of an LLF/HLL solver), for
    lambda = max(|v_n| + c) whenever every wave lies inside the fan (for a strong
    shock such as Sod's it need not: that speed is no bound on the fan)."""
    WL, WR = RIEMANN[case]
    uL, uR = _cons(*WL), _cons(*WR)
    if d == 1:  # same problem along y: swap the velocity components
        uL, uR = uL[[0, 2, 1, 3]], uR[[0, 2, 1, 3]]
    cL, cR = np.sqrt(G * WL[3] / WL[0]), np.sqrt(G * WR[3] / WR[0])
    lam = max(abs(WL[1]) + cL, abs(WR[1]) + cR)
    ref, smax = _fan_average(uL, uR, d, lam, G)
    assert smax <= lam * (1 + 1e-14)  # the fan lies inside [-lam, lam]
    ub = oracle.bar_state(uL, uR, d, G)
    assert np.abs(ub - ref).max() < 1e-12 * np.abs(ref).max(), (ub, ref)


def _bounds_from_edges(oracle, M, u):
    lo = u[:, 0].copy()
    hi = u[:, 0].copy()
    sm = np.zeros_like(lo)
    for e in range(M.E):
        for b in range(M.n):
            for a in range(M.n):
                sm[e, b, a] = oracle.spec_entropy(u[e, :, b, a], G)
    for (e, a, b, e2, a2, b2, d, sgn, c) in _edges(M, oracle):
        ui, uj = u[e, :, b, a], u[e2, :, b2, a2]
        ub = oracle.bar_state(ui, uj, d, G) if sgn > 0 else oracle.bar_state(uj, ui, d, G)
        lo[e, b, a] = min(lo[e, b, a], ub[0])
        hi[e, b, a] = max(hi[e, b, a], ub[0])
        sm[e, b, a] = min(sm[e, b, a], oracle.spec_entropy(ub, G))
    return lo, hi, sm


@pytest.mark.parametrize("N,seed", [(3, 0), (3, 3), (4, 1)])
def test_local_bounds_over_the_low_order_graph(oracle, N, seed):
    """The oracle's bounds are the min / max over the node and the bar states of
    its low-order graph neighbours, the graph being the one whose bar-state form
    reproduces the low-order residual (eq. barstateform)."""
    M = make(oracle, random_mesh(seed, 4, 3, 0.4), N)
    x, y, m = M.geometry()
    u = states.random_admissible(x, 40 + seed)
    lo, hi, sm = M.local_bounds(u)
    rlo, rhi, rsm = _bounds_from_edges(oracle, M, u)
    assert np.array_equal(lo, rlo) and np.array_equal(hi, rhi) and np.array_equal(sm, rsm)
    assert M.M > 0


@pytest.mark.parametrize("seed", range(3))
def test_low_order_state_within_local_bounds(oracle, seed):
    """Under the IDP time step the low-order update is a convex combination of the
    node and its bar states (eq. convex_combination), so it meets the local density
    bounds and, p rho^-gamma being quasi-concave, the entropy bound; at three times
    that step it leaves them somewhere (the bounds are not vacuous)."""
    M = make(oracle, random_mesh(seed, 4, 3, 0.4))
    x, y, m = M.geometry()
    u = states.random_admissible(x, 60 + seed)
    lo, hi, sm = M.local_bounds(u)
    for cfl, inside in ((1.0, True), (0.5, True), (3.0, False)):
        dt = M.max_dt(u, cfl)
        uf = u + dt * M.rhs(u, oracle.RHS_LOW)
        s = np.array([oracle.spec_entropy(uf[e, :, b, a], G) for e in range(M.E)
                      for b in range(M.n) for a in range(M.n)]).reshape(lo.shape)
        ok = ((uf[:, 0] >= lo * (1 - 1e-13)) & (uf[:, 0] <= hi * (1 + 1e-13)) &
              (s >= sm * (1 - 1e-12)))
        assert ok.all() == inside, (cfl, (~ok).sum())


def test_theta_entropy_against_bisection(oracle):
    """Largest theta in [0, thi] with p rho^-gamma >= st along the ray, against
    bisection on the entropy itself; the returned state is feasible."""
    rng = np.random.default_rng(7)
    n_root = 0
    for _ in range(300):
        w0 = (rng.uniform(0.2, 2), rng.uniform(-1, 1), rng.uniform(-1, 1), rng.uniform(0.1, 2))
        u0 = _cons(*w0)
        dc = rng.normal(size=4) * np.array([0.3, 0.3, 0.3, 0.6])
        s0 = oracle.spec_entropy(u0, G)
        st = s0 * rng.uniform(0.5, 1.0)
        thi = rng.choice([1.0, rng.uniform(0.1, 1.0)])
        # keep the ray inside rho > 0 and p > 0 up to thi
        for _ in range(60):
            q = u0 + thi * dc
            if q[0] > 0 and oracle.spec_entropy(q, G) > 0:
                break
            thi *= 0.5
        th = oracle.theta_entropy(u0, dc, st, G, thi)
        assert 0.0 <= th <= thi

        def feas(t):
            return oracle.spec_entropy(u0 + t * dc, G) >= st
        if feas(thi):
            assert th == thi
            continue
        lo_, hi_ = 0.0, thi
        for _ in range(200):
            mid = 0.5 * (lo_ + hi_)
            lo_, hi_ = (mid, hi_) if feas(mid) else (lo_, mid)
        assert abs(th - lo_) < 1e-12, (th, lo_)
        assert oracle.spec_entropy(u0 + th * dc, G) >= st * (1 - 1e-14)
        n_root += 1
    assert n_root > 50
    # an infeasible start gives 0
    u0 = _cons(1.0, 0.0, 0.0, 1.0)
    assert oracle.theta_entropy(u0, np.array([0.1, 0, 0, -0.5]), 1.01, G, 1.0) == 0.0


@pytest.mark.parametrize("seed", [0, 1])
def test_local_limiting_blast_bounds_and_conservation(oracle, seed):
    """Local limiting on a blast over a refined mesh with mortars: every node stays
    inside its bounds after each stage, and mass, momentum and energy are conserved
    to rounding (one factor per subcell face and per mortar)."""
    M = make(oracle, random_mesh(seed, 4, 3, 0.4))
    x, y, m = M.geometry()
    u = states.sedov_gaussian(2 * x - 1, 2 * y - 1, sigma=0.15)
    tot0 = (u * m[:, None]).sum(axis=(0, 2, 3))
    limited = 1.0
    for _ in range(5):
        u, st = M.ssprk3(u, 0.5, limiter=oracle.LIM_LOCAL)
        assert st["violations"] == 0 and st["fv_inadmissible"] == 0
        limited = min(limited, st["theta_vol_min"], st["theta_mort_min"])
    tot = (u * m[:, None]).sum(axis=(0, 2, 3))
    scale = (np.abs(u) * m[:, None]).sum(axis=(0, 2, 3))
    assert np.all(np.abs(tot - tot0) < 1e-13 * scale)
    assert limited < 0.5


def test_local_limiting_free_stream(oracle):
    """A constant state stays constant to rounding under local limiting."""
    M = make(oracle, random_mesh(2, 4, 3, 0.4))
    x, y, m = M.geometry()
    u = states.constant(x, rho=1.1, v1=0.3, v2=-0.2, p=0.8)
    v, st = M.ssprk3(u, 0.5, limiter=oracle.LIM_LOCAL)
    assert np.abs(v - u).max() < 1e-13 * np.abs(u).max()
    assert st["violations"] == 0


def _density_wave_local(oracle, N, lev):
    ms = refined_box_mesh(2 ** lev, (-0.5, -0.5), (0.0, 0.5), -1.0, -1.0, 2.0)
    M = make(oracle, ms, N)
    x, y, m = M.geometry()
    u = states.density_wave(x, y)
    t, viol = 0.0, 0
    while t < 1.0 - 1e-14:
        dt = min(M.max_dt(u, 0.95), 1.0 - t)
        u, st = M.ssprk3_dt(u, dt, limiter=oracle.LIM_LOCAL)
        t += dt
        viol += st["violations"]
    err = _l2_errors(oracle, M, u, lambda xx, yy: states.density_wave(xx, yy, t=1.0), 4.0)
    return err, viol


def test_density_wave_local_limiting_paper_table(oracle):
    """Table ConvergenceTestLocalLimiting, N = 3, levels 2 and 3: the limiter now
    acts on the smooth wave and the errors are those of a first-order-like scheme.
    The oracle's errors lie 14% and 7% below the printed ones; the gap closes with
    refinement (2% at level 4, the slow test, and 0.5% at level 5: 0.03353 against
    0.0337, EOC 1.00 against 1.03, measured once); the EOC, the variable ratios
    0.1 : 0.2 : 0.025 (velocity and pressure stay constant) and the bounds hold.
    The gap halves per level like the share of mortar nodes: with every mortar
    forced to its low-order flux the oracle gives 0.5345 and 0.1746 (printed
    0.543 and 0.169), so the printed runs limit the mortars far more strongly
    than the oracle's mean mortar alpha of about 0.05 (measured once, on copies
    of the oracle)."""
    tab = T["density_wave_local"]["3"]
    errs = []
    for lev, tol in ((2, 0.16), (3, 0.09)):
        err, viol = _density_wave_local(oracle, 3, lev)
        ref = np.array(tab[str(lev)])
        assert np.all(np.abs(err - ref) <= tol * ref), (lev, err, ref)
        assert np.allclose(err[1:] / err[0], [0.1, 0.2, 0.025], rtol=1e-6)
        assert viol == 0
        errs.append(err[0])
    eoc = np.log(errs[0] / errs[1]) / np.log(2)
    assert abs(eoc - T["density_wave_local"]["eoc"]["3"]["3"]) < 0.15
    # far above the positivity-limited errors of the same meshes
    assert errs[0] > 5 * T["density_wave_positivity"]["3"]["2"][0]


@pytest.mark.slow
def test_density_wave_local_limiting_level4(oracle):
    err, viol = _density_wave_local(oracle, 3, 4)
    ref = np.array(T["density_wave_local"]["3"]["4"])
    assert np.all(np.abs(err - ref) <= 0.03 * ref) and viol == 0
