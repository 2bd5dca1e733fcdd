"""Pins of the oracle's semi-discretisation, time step, limiter and SSP-RK3 against
properties the paper proves and values it prints."""
import numpy as np
import pytest

from paper_values import tables
from workloads import states
from workloads.meshes import workload_mesh, random_mesh, refined_box_mesh, uniform_mesh

T = tables()


def make(oracle, spec, N=3):
    return oracle.Mesh(N, *spec.args())


MESHES = {
    "vortex304": lambda: workload_mesh("vortex304"),
    "random0": lambda: random_mesh(0, 4, 3, 0.4),
    "random3": lambda: random_mesh(3, 4, 3, 0.4),
    "uniform": lambda: uniform_mesh(5, 3, Lx=1.0, Ly=0.6),
}


@pytest.mark.parametrize("name", sorted(MESHES))
@pytest.mark.parametrize("N", [3, 4])
def test_free_stream_and_conservation(oracle, name, N):
    """A constant state is preserved (u_dot = 0) and sum_i m_i u_dot_i = 0 for both
    schemes, with and without mortars (eq. conservationProperty)."""
    M = make(oracle, MESHES[name](), N)
    x, y, m = M.geometry()
    u = states.constant(x)
    for which in (oracle.RHS_HIGH, oracle.RHS_LOW):
        du = M.rhs(u, which)
        assert np.abs(du).max() < 1e-12 * (1.0 / m.min() ** 0.5)
    # per-node noise small enough that mortar interpolation stays admissible
    u = states.random_admissible(x, 7, rho_range=(0.8, 1.2), p_range=(0.8, 1.2), vmax=0.3)
    for which in (oracle.RHS_HIGH, oracle.RHS_LOW):
        du = M.rhs(u, which)
        total = (du * m[:, None]).sum(axis=(0, 2, 3))
        scale = (np.abs(du) * m[:, None]).sum(axis=(0, 2, 3))
        assert np.all(np.abs(total) < 1e-14 * scale)


def _edges(M, oracle):
    """Low-order graph of eq. LowOrderScheme_globalIndices built from the paper's
    c_ij (Sec. 2.1) and the sparse mortar c_ij = tilde-omega n / 2 (eq. c_nonconforming):
    yields (e, a, b, e2, a2, b2, dir, sign, |c|)."""
    N, n = M.N, M.n
    xi, w, D, S = oracle.basis(N)
    I, P, W = oracle.mortar_ops(N)
    faces, morts = M.faces(), M.mortars()
    x0, y0, Lx, Ly, nx0, ny0 = M.box
    hx = Lx / (nx0 * 2.0 ** M.level.astype(float))
    hy = Ly / (ny0 * 2.0 ** M.level.astype(float))

    def fnode(f, k):
        return [(0, k), (N, k), (k, 0), (k, N)][f]

    out = []
    for e in range(M.E):
        for b in range(n):
            for a in range(n):
                if a > 0: out.append((e, a, b, e, a - 1, b, 0, -1, w[b] * hy[e] / 4))
                if a < N: out.append((e, a, b, e, a + 1, b, 0, +1, w[b] * hy[e] / 4))
                if b > 0: out.append((e, a, b, e, a, b - 1, 1, -1, w[a] * hx[e] / 4))
                if b < N: out.append((e, a, b, e, a, b + 1, 1, +1, w[a] * hx[e] / 4))
                for f in range(4):
                    if fnode(f, a if f >= 2 else b) != (a, b):
                        continue
                    k = a if f >= 2 else b
                    typ, nbr, mort, half = faces[e, f]
                    d, sgn = f // 2, (1 if f % 2 else -1)
                    hf = hy[e] if f < 2 else hx[e]
                    if typ == 0:
                        a2, b2 = fnode(f ^ 1, k)
                        out.append((e, a, b, nbr, a2, b2, d, sgn, w[k] * hf / 4))
                    elif typ == 2:
                        L, fl, s0, s1 = morts[mort]
                        for h, s in ((0, s0), (1, s1)):
                            for l in range(n):
                                if W[k, h * n + l] > 0:
                                    a2, b2 = fnode(f ^ 1, l)
                                    out.append((e, a, b, s, a2, b2, d, sgn, W[k, h * n + l] * hf / 4))
                    else:
                        L, fl, s0, s1 = morts[mort]
                        hL = 2 * hf
                        for kk in range(n):
                            if W[kk, half * n + k] > 0:
                                a2, b2 = fnode(fl, kk)
                                out.append((e, a, b, L, a2, b2, d, sgn, W[kk, half * n + k] * hL / 4))
    return out


def _phys(u, d, g):
    rho = u[0]
    v = u[1:3] / rho
    p = (g - 1) * (u[3] - 0.5 * rho * (v @ v))
    vn = v[d]
    f = np.array([rho * vn, u[1] * vn, u[2] * vn, (u[3] + p) * vn])
    f[1 + d] += p
    return f, abs(vn) + np.sqrt(g * p / rho)


@pytest.mark.parametrize("name", ["random0", "vortex304"])
def test_low_order_bar_state_form(oracle, name):
    """m_i u_dot_i = sum_j 2 d_ij (ubar_ij - u_i) (eq. barstateform), evaluated from
    the paper's bar states, equals the oracle's low-order residual; also checks
    dt <= m_i / sum 2 d_ij (eq. timestep_restriction) against the oracle's dt."""
    g = 1.4
    M = make(oracle, MESHES[name]())
    x, y, m = M.geometry()
    u = states.random_admissible(x, 21)
    R = M.rhs(u, oracle.RHS_LOW) * m[:, None]
    ref = np.zeros_like(R)
    dsum = np.zeros_like(m)
    for (e, a, b, e2, a2, b2, d, sgn, c) in _edges(M, oracle):
        ui, uj = u[e, :, b, a], u[e2, :, b2, a2]
        fi, li = _phys(ui, d, g)
        fj, lj = _phys(uj, d, g)
        dij = c * max(li, lj)
        ubar = 0.5 * (ui + uj) - sgn * c * (fj - fi) / (2 * dij)
        ref[e, :, b, a] += 2 * dij * (ubar - ui)
        dsum[e, b, a] += 2 * dij
    scale = np.abs(ref).max()
    assert np.abs(R - ref).max() < 1e-13 * scale
    dt_ref = (m / dsum).min()
    assert abs(M.max_dt(u, 1.0) - dt_ref) < 1e-14 * dt_ref


def test_dt_closed_form_uniform(oracle):
    """Uniform mesh, constant state: the IDP bound is
    1 / (4 (lambda_x / (hx w_0) + lambda_y / (hy w_0))) at a corner node."""
    g, N = 1.4, 3
    M = make(oracle, uniform_mesh(6, 4, Lx=1.2, Ly=0.4), N)
    x, y, m = M.geometry()
    u = states.constant(x, rho=1.3, v1=0.4, v2=-0.7, p=0.9)
    xi, w, D, S = oracle.basis(N)
    c = np.sqrt(g * 0.9 / 1.3)
    hx, hy = 0.2, 0.1
    ref = 1.0 / (4 * ((0.4 + c) / (hx * w[0]) + (0.7 + c) / (hy * w[0])))
    assert abs(M.max_dt(u, 1.0) - ref) < 1e-14 * ref
    assert abs(M.max_dt(u, 0.5) - 0.5 * ref) < 1e-14 * ref
    lo = 1.0 / ((N + 1) * ((0.4 + c) / hx + (0.7 + c) / hy))
    assert abs(M.max_dt(u, 1.0, oracle.DT_LOWORDER) - lo) < 1e-14 * lo


def test_low_order_step_positive_near_vacuum(oracle):
    """Under the IDP time step the low-order update is a convex combination of
    bar states (eq. convex_combination), hence stays admissible even near vacuum."""
    M = make(oracle, random_mesh(2, 4, 3, 0.4))
    x, y, m = M.geometry()
    for seed in range(3):
        u = states.random_admissible(x, 100 + seed, rho_range=(1e-8, 2.0),
                                     p_range=(1e-12, 3.0), vmax=3.0)
        dt = M.max_dt(u, 1.0)
        uf = u + dt * M.rhs(u, oracle.RHS_LOW)
        rho = uf[:, 0]
        p = 0.4 * (uf[:, 3] - 0.5 * (uf[:, 1] ** 2 + uf[:, 2] ** 2) / uf[:, 0])
        assert (rho > 0).all() and (p > 0).all()


def test_limiter_inactive_on_smooth_flow_equals_high_order(oracle):
    """Far from the bounds nothing is limited and the limited step equals the
    high-order step (Sec. 3.1: results without limiting are identical); this also
    ties the telescoped subcell fluxes (eq. fluxdifferencingform) to the direct
    volume term."""
    M = make(oracle, random_mesh(1, 4, 3, 0.4))
    x, y, m = M.geometry()
    u = states.density_wave(x, y)
    dt = M.max_dt(u, 0.9)
    a, sa = M.fe_step(u, dt, limiter=oracle.LIM_POSITIVITY)
    b, sb = M.fe_step(u, dt, limiter=oracle.LIM_NONE)
    assert sa["theta_vol_min"] == 1.0 and sa["theta_mort_min"] == 1.0
    assert np.abs(a - b).max() < 1e-13 * np.abs(u).max()


def _l2_errors(oracle, M, u, exact_fn, area):
    """L2 error with the solution interpolated to degree-2N LGL points per direction."""
    from numpy.polynomial import legendre as npleg
    N = M.N
    xi, _, _, _ = oracle.basis(N)
    Na = 2 * N
    c = np.zeros(Na + 1)
    c[Na] = 1
    xa = np.concatenate(([-1.0], np.sort(npleg.legroots(npleg.legder(c))), [1.0]))
    wa = 2.0 / (Na * (Na + 1) * npleg.legval(xa, c) ** 2)
    V = np.array([[oracle.lagrange(N, k, s) for k in range(N + 1)] for s in xa])
    x, y, m = M.geometry()

    def up(f):
        f = np.einsum("ik,...jk->...ji", V, f)
        return np.einsum("jl,...li->...ji", V, f)
    J = m.sum(axis=(1, 2)) / 4.0
    err = up(u) - exact_fn(up(x), up(y))
    return np.sqrt(np.einsum("evji,j,i,e->v", err ** 2, wa, wa, J) / area)


def _density_wave_run(oracle, N, lev):
    ms = refined_box_mesh(2 ** lev, (-0.5, -0.5), (0.0, 0.5), -1.0, -1.0, 2.0)
    M = make(oracle, ms, N)
    x, y, m = M.geometry()
    u = states.density_wave(x, y)
    t, Tend, viol, thmin = 0.0, 1.0, 0, 1.0
    while t < Tend - 1e-14:
        dt = min(M.max_dt(u, 0.95), Tend - t)
        u, st = M.ssprk3_dt(u, dt)
        t += dt
        viol += st["violations"]
        thmin = min(thmin, st["theta_vol_min"], st["theta_mort_min"])
    err = _l2_errors(oracle, M, u, lambda xx, yy: states.density_wave(xx, yy, t=Tend), 4.0)
    return err, viol, thmin


@pytest.mark.parametrize("N,levels", [(3, (2, 3)), (4, (2, 3))])
def test_density_wave_matches_paper_table(oracle, N, levels):
    """Table ConvergenceTestPositivity (N=3) and Table ConvergenceTest_polydeg4 (N=4):
    the printed errors (3 significant digits), the EOC, the exact 0.1 : 0.2 : 0.025
    ratios between the variables' errors, and no limiting at all."""
    tab = T["density_wave_positivity"][str(N)]
    errs = []
    for lev in levels:
        err, viol, thmin = _density_wave_run(oracle, N, lev)
        ref = np.array(tab[str(lev)])
        assert np.all(np.abs(err - ref) <= 0.005 * ref + 1e-16), (lev, err, ref)
        assert np.allclose(err[1:] / err[0], [0.1, 0.2, 0.025], rtol=1e-6)
        assert viol == 0 and thmin == 1.0
        errs.append(err[0])
    eoc = np.log(errs[0] / errs[1]) / np.log(2)
    assert abs(eoc - T["density_wave_positivity"]["eoc"][str(N)][str(levels[1])]) < 0.01


@pytest.mark.slow
def test_density_wave_level4(oracle):
    err, viol, thmin = _density_wave_run(oracle, 3, 4)
    ref = np.array(T["density_wave_positivity"]["3"]["4"])
    assert np.all(np.abs(err - ref) <= 0.005 * ref)


def _isentropic_exact(x, y, t, g=3.0):
    s2 = np.sqrt(2.0)

    def rho0(z):
        return 1.0 + 0.9999999 * np.sin(np.pi * z)
    xp = (x + y) / s2

    def solve(sgn):
        z = xp.copy()
        for _ in range(60):
            F = xp + sgn * np.sqrt(3) * rho0(z) * t - z
            dF = sgn * np.sqrt(3) * 0.9999999 * np.pi * np.cos(np.pi * z) * t - 1.0
            z = z - F / dF
        return z
    x1, x2 = solve(1.0), solve(-1.0)
    rho = 0.5 * (rho0(x1) + rho0(x2))
    vth = np.sqrt(3) * (rho - rho0(x1))
    return states.conservative(rho, vth / s2, vth / s2, rho ** g, g)


def test_isentropic_flow_matches_paper_table(oracle):
    """Table ConvergenceTestIsentropicFlow, N=3, levels 2..4: near-vacuum flow where the
    positivity limiter is active in the volume and at the mortars; errors within 2.5%
    of the printed values, zero bound violations, admissible low-order states."""
    g, s2 = 3.0, np.sqrt(2.0)
    tab = T["isentropic_flow"]["3"]
    for lev in (2, 3, 4):
        ms = refined_box_mesh(2 ** lev, (-1 / s2, -1 / s2), (0.0, 1 / s2), -s2, -s2, 2 * s2)
        M = make(oracle, ms, 3)
        x, y, m = M.geometry()
        u = states.isentropic_flow(x, y, gamma=g)
        t, Tend, viol, inad, thmin = 0.0, 0.1, 0, 0, 1.0
        while t < Tend - 1e-14:
            dt = min(M.max_dt(u, 0.5, oracle.DT_LOWORDER, gamma=g), Tend - t)
            u, st = M.ssprk3_dt(u, dt, gamma=g)
            t += dt
            viol += st["violations"]
            inad += st["fv_inadmissible"]
            thmin = min(thmin, st["theta_vol_min"])
        err = _l2_errors(oracle, M, u, lambda xx, yy: _isentropic_exact(xx, yy, Tend), 8.0)
        ref = np.array(tab[str(lev)])
        assert np.all(np.abs(err - ref) <= 0.025 * ref), (lev, err, ref)
        assert viol == 0 and inad == 0
        assert thmin < 0.01  # the limiter is active


def test_ssprk3_third_order_in_time(oracle):
    """Halving dt on a fixed mesh divides the time error by about 8 (Shu-Osher SSP-RK3)."""
    M = make(oracle, refined_box_mesh(4, (-0.5, -0.5), (0.0, 0.5), -1.0, -1.0, 2.0), 3)
    x, y, m = M.geometry()
    u0 = states.density_wave(x, y)

    def run(dt, Tend=0.08):
        u = u0.copy()
        for _ in range(int(round(Tend / dt))):
            u, _ = M.ssprk3_dt(u, dt, limiter=oracle.LIM_NONE)
        return u
    ref = run(0.00025)
    e1 = np.abs(run(0.004) - ref).max()
    e2 = np.abs(run(0.002) - ref).max()
    assert 6.5 < e1 / e2 < 9.5


def test_theta_pressure_brute_force(oracle):
    """The pressure factor is the largest admissible theta along the ray: scan
    theta on a fine grid (Q: a root of p(u0 + theta dc) = p_min)."""
    g = 1.4
    rng = np.random.default_rng(5)
    for _ in range(200):
        rho, v1, v2, p = rng.uniform(0.1, 2), rng.normal(), rng.normal(), rng.uniform(0.05, 2)
        u0 = states.conservative(np.array([rho]), np.array([v1]), np.array([v2]),
                                 np.array([p]), g)[0]
        dc = rng.normal(size=4) * rng.uniform(0.1, 3) * np.array([rho, rho, rho, p])
        pt = 0.1 * p
        th = oracle.theta_pressure(u0, dc, pt, g)
        grid = np.linspace(0, 1, 20001)
        U = u0[None, :] + grid[:, None] * dc[None, :]
        pp = (g - 1) * (U[:, 3] - 0.5 * (U[:, 1] ** 2 + U[:, 2] ** 2) / U[:, 0])
        ok = (U[:, 0] > 0) & (pp >= pt)
        bad = np.nonzero(~ok)[0]
        ref = 1.0 if len(bad) == 0 else grid[bad[0]]
        assert ref - 6e-5 <= th <= ref + 1e-12, (th, ref)
        if th < 1:
            u = u0 + th * dc
            pth = (g - 1) * (u[3] - 0.5 * (u[1] ** 2 + u[2] ** 2) / u[0])
            assert abs(pth - pt) < 1e-9 * (abs(u[3]) + p)


@pytest.mark.parametrize("seed", [0, 1])
def test_blast_positivity_and_conservation(oracle, seed):
    """Top-hat blast (Sec. 3.4 initial state) on a 2:1 mesh: the limiter acts in the
    volume and at the mortars, all bounds hold, mass/momentum/energy are conserved."""
    spec = random_mesh(10 + seed, 8, 2, 0.45, L=4.0, x0=-2.0, y0=-2.0)
    M = make(oracle, spec)
    x, y, m = M.geometry()
    u = states.sedov_tophat(x, y, r0=0.5)
    tot0 = (u * m[:, None]).sum(axis=(0, 2, 3))
    thmin, tmmin = 1.0, 1.0
    for _ in range(8):
        u, st = M.ssprk3(u, 0.9)
        assert st["violations"] == 0 and st["fv_inadmissible"] == 0
        thmin = min(thmin, st["theta_vol_min"])
        tmmin = min(tmmin, st["theta_mort_min"])
    tot = (u * m[:, None]).sum(axis=(0, 2, 3))
    assert np.all(np.abs(tot - tot0) <= 1e-13 * np.abs(u * m[:, None]).sum(axis=(0, 2, 3)))
    assert thmin < 0.5
    assert (u[:, 0] > 0).all()
