/*
 * Oracle: semi-discretisation, time-step restriction, limited forward-Euler
 * step and SSP-RK3.  TEST INFRASTRUCTURE ONLY (see dgo.h).
 *
 * All residuals here are R_i = m_i du_i/dt with the mass m_i = J omega_a omega_b,
 * J = hx hy / 4 (eq. evolutionformula).
 *
 *  High order (eq. evolutionformula and the volume term F^Vol below it):
 *    R_ab = omega_b ( -sum_k Sbar_ak (hy/2) f*_x(u_ab, u_kb) + boundary fluxes )
 *         + omega_a ( -sum_k Sbar_bk (hx/2) f*_y(u_ab, u_ak) + boundary fluxes )
 *    with LLF surface fluxes on conforming faces and Kopriva's L2 mortar
 *    (interpolate, LLF on the mortar = small face, project back) on mortars.
 *  Low order (eq. FVmethod, eq. interfaceflux_local):
 *    LLF subcell fluxes between neighbouring nodes; on conforming faces the same
 *    LLF as above; on mortars the sparsified IDP flux with weights tilde-omega.
 *  Time step (eq. timestep_restriction; eq. CFLcondition_lowordermethod).
 *  Limiting (Sec. 2.3): low-order update, then the volume correction with one
 *  factor per subcell face, then the mortar correction with one factor per
 *  mortar, against the positivity bounds of eq. Bounds_Positivity, and with
 *  local limiting also against the bar-state bounds of eq. Bounds_Barstates
 *  (density minimum and maximum, minimum of the specific entropy), and with
 *  combined limiting (eq. combination_posLim_local) both factor sets blended
 *  per element by a shock indicator on the pressure.
 *  Time integration: three-stage SSP Runge-Kutta (Shu & Osher 1988, Sec. 3).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "dgo.h"

#define IDX(e, v, b, a) ((((int64_t)(e)*4 + (v)) * n + (b)) * n + (a))

/* node (a, b) of element face f at position k along the face */
static void face_node(int f, int k, int N, int* a, int* b)
{
    if (f == 0) { *a = 0; *b = k; }
    else if (f == 1) { *a = N; *b = k; }
    else if (f == 2) { *a = k; *b = 0; }
    else { *a = k; *b = N; }
}

static void get_node(const double* u, int n, int64_t e, int a, int b, double* q)
{
    for (int v = 0; v < 4; ++v) q[v] = u[IDX(e, v, b, a)];
}

static double face_len(const dgo_mesh* m, int64_t e, int f) { return f < 2 ? m->hy[e] : m->hx[e]; }

/* ---------------------------------------------------------------------------
 * Mortar contributions.  For mortar S, slot s in [0, 3n): s < n is large-face
 * node k = s; s = n + h n + l is node l of small element h.  HO[S][s][v] and
 * LO[S][s][v] are the mortar's contributions to R of that node.
 * ------------------------------------------------------------------------- */
static void mortar_contrib(const dgo_mesh* m, const double* u, double gamma, int64_t S, double* HO,
                           double* LO)
{
    const dgo_basis* B = &m->B;
    int N = B->N, n = B->n;
    const dgo_mortar* M = &m->mort[S];
    int f = M->face, dir = f / 2;
    int large_lower = (f & 1); /* large element sits on the low-coordinate side */
    double sgn_large = large_lower ? -1.0 : 1.0, sgn_small = -sgn_large;
    double hL = face_len(m, M->large, f), hs = 0.5 * hL;
    double uL[DGO_NMAX][4], us[2][DGO_NMAX][4];
    for (int k = 0; k < n; ++k) {
        int a, b;
        face_node(f, k, N, &a, &b);
        get_node(u, n, M->large, a, b, uL[k]);
    }
    for (int h = 0; h < 2; ++h)
        for (int l = 0; l < n; ++l) {
            int a, b;
            face_node(f ^ 1, l, N, &a, &b);
            get_node(u, n, M->small[h], a, b, us[h][l]);
        }
    for (int s = 0; s < 3 * n; ++s)
        for (int v = 0; v < 4; ++v) HO[s * 4 + v] = LO[s * 4 + v] = 0.0;

    /* high order: L2 mortar */
    double Fm[2][DGO_NMAX][4];
    for (int h = 0; h < 2; ++h)
        for (int l = 0; l < n; ++l) {
            double ui[4] = {0, 0, 0, 0};
            for (int k = 0; k < n; ++k)
                for (int v = 0; v < 4; ++v) ui[v] += B->I[h][l][k] * uL[k][v];
            /* an interpolated state outside the admissible set leaves the
               high-order mortar flux undefined (Sec. 3.2): mark it NaN, the
               mortar limiter then keeps the low-order flux */
            if (!(ui[0] > 0.0) || !(dgo_pressure(ui, gamma) > 0.0)) {
                for (int v = 0; v < 4; ++v) Fm[h][l][v] = NAN;
            } else if (large_lower) {
                dgo_flux_llf(ui, us[h][l], dir, gamma, Fm[h][l]);
            } else {
                dgo_flux_llf(us[h][l], ui, dir, gamma, Fm[h][l]);
            }
            for (int v = 0; v < 4; ++v)
                HO[(n + h * n + l) * 4 + v] = sgn_small * B->w[l] * hs / 2.0 * Fm[h][l][v];
        }
    for (int k = 0; k < n; ++k)
        for (int v = 0; v < 4; ++v) {
            double pk = 0.0;
            for (int h = 0; h < 2; ++h)
                for (int l = 0; l < n; ++l) pk += B->P[h][k][l] * Fm[h][l][v];
            HO[k * 4 + v] = sgn_large * B->w[k] * hL / 2.0 * pk;
        }

    /* low order: sparse IDP mortar flux */
    for (int k = 0; k < n; ++k)
        for (int h = 0; h < 2; ++h)
            for (int l = 0; l < n; ++l) {
                double wt = B->Wt[k][h * n + l];
                if (wt == 0.0) continue;
                double W = wt * hL / 2.0, G[4];
                if (large_lower) dgo_flux_llf(uL[k], us[h][l], dir, gamma, G);
                else dgo_flux_llf(us[h][l], uL[k], dir, gamma, G);
                for (int v = 0; v < 4; ++v) {
                    LO[k * 4 + v] += sgn_large * W * G[v];
                    LO[(n + h * n + l) * 4 + v] += sgn_small * W * G[v];
                }
            }
}

static int is_mortar(int type) { return type == FACE_SMALL || type == FACE_LARGE; }

/* slot of node k along face f of element e, or -1 if that face is not a mortar */
static int64_t face_slot(const dgo_mesh* m, int64_t e, int f, int k)
{
    const dgo_face* F = &m->face[e * 4 + f];
    int n = m->B.n;
    if (F->type == FACE_LARGE) return F->mortar * 3 * n + k;
    if (F->type == FACE_SMALL) return F->mortar * 3 * n + n + F->half * n + k;
    return -1;
}

/* the state across face f at node k of element e, whose own state is ui: the
   matching node of the neighbour (conforming face) or the ghost state of the
   node's boundary condition (boundary face) */
static void across_node(const dgo_mesh* m, const double* u, double gamma, int64_t e, int f, int k,
                        const double* ui, double* uo)
{
    const dgo_face* F = &m->face[e * 4 + f];
    if (F->type == FACE_BOUNDARY) {
        int64_t j = F->bnode + k;
        dgo_boundary_ghost(m->bkind[j], m->bext + j * 4, ui, f, gamma, uo);
        return;
    }
    int a2, b2;
    face_node(f ^ 1, k, m->B.N, &a2, &b2);
    get_node(u, m->B.n, F->nbr, a2, b2, uo);
}

/* conforming or boundary face contribution to R of node k of face f of element e */
static void conf_face(const dgo_mesh* m, const double* u, double gamma, int64_t e, int f, int k,
                      double* r)
{
    const dgo_basis* B = &m->B;
    int N = B->N, n = B->n;
    int a, b;
    face_node(f, k, N, &a, &b);
    double ui[4], uo[4], Fl[4];
    get_node(u, n, e, a, b, ui);
    across_node(m, u, gamma, e, f, k, ui, uo);
    int dir = f / 2;
    double W = B->w[k] * face_len(m, e, f) / 2.0;
    if (f & 1) { /* element on the low side */
        dgo_flux_llf(ui, uo, dir, gamma, Fl);
        for (int v = 0; v < 4; ++v) r[v] = -W * Fl[v];
    } else {
        dgo_flux_llf(uo, ui, dir, gamma, Fl);
        for (int v = 0; v < 4; ++v) r[v] = W * Fl[v];
    }
}

/* surface contributions (conforming faces and mortar slots) for element e */
static void add_surface(const dgo_mesh* m, const double* u, double gamma, const double* slots,
                        int64_t e, double* R /* [4][n][n] */)
{
    int N = m->B.N, n = m->B.n;
    for (int f = 0; f < 4; ++f) {
        const dgo_face* F = &m->face[e * 4 + f];
        for (int k = 0; k < n; ++k) {
            int a, b;
            face_node(f, k, N, &a, &b);
            double r[4];
            if (F->type == FACE_CONF || F->type == FACE_BOUNDARY) {
                conf_face(m, u, gamma, e, f, k, r);
            } else {
                int64_t s = face_slot(m, e, f, k);
                for (int v = 0; v < 4; ++v) r[v] = slots[s * 4 + v];
            }
            for (int v = 0; v < 4; ++v) R[(v * n + b) * n + a] += r[v];
        }
    }
}

static void compute_slots(const dgo_mesh* m, const double* u, double gamma, double* HO, double* LO)
{
    int n = m->B.n;
#pragma omp parallel for schedule(static)
    for (int64_t S = 0; S < m->M; ++S)
        mortar_contrib(m, u, gamma, S, HO + S * 3 * n * 4, LO + S * 3 * n * 4);
}

/* high-order volume term, direct sum form */
static void volume_high(const dgo_mesh* m, const double* u, double gamma, int64_t e, double* R)
{
    const dgo_basis* B = &m->B;
    int n = B->n;
    double hx = m->hx[e], hy = m->hy[e];
    for (int b = 0; b < n; ++b)
        for (int a = 0; a < n; ++a) {
            double ui[4], uk[4], fs[4], acc[4] = {0, 0, 0, 0};
            get_node(u, n, e, a, b, ui);
            for (int k = 0; k < n; ++k) {
                get_node(u, n, e, k, b, uk);
                dgo_flux_volume(m->vflux, ui, uk, 0, gamma, fs);
                for (int v = 0; v < 4; ++v) acc[v] -= B->w[b] * B->S[a][k] * (hy / 2.0) * fs[v];
                get_node(u, n, e, a, k, uk);
                dgo_flux_volume(m->vflux, ui, uk, 1, gamma, fs);
                for (int v = 0; v < 4; ++v) acc[v] -= B->w[a] * B->S[b][k] * (hx / 2.0) * fs[v];
            }
            for (int v = 0; v < 4; ++v) R[(v * n + b) * n + a] += acc[v];
        }
}

/* low-order FV subcell fluxes, scaled subcell LLF flux on each interior subcell face */
static void fv_face_flux(const dgo_mesh* m, const double* u, double gamma, int64_t e, int dir,
                         int line, int a, double* F)
{
    int n = m->B.n;
    double q0[4], q1[4];
    if (dir == 0) {
        get_node(u, n, e, a, line, q0);
        get_node(u, n, e, a + 1, line, q1);
    } else {
        get_node(u, n, e, line, a, q0);
        get_node(u, n, e, line, a + 1, q1);
    }
    dgo_flux_llf(q0, q1, dir, gamma, F);
    double s = (dir == 0 ? m->hy[e] : m->hx[e]) / 2.0;
    for (int v = 0; v < 4; ++v) F[v] *= s;
}

static void volume_low(const dgo_mesh* m, const double* u, double gamma, int64_t e, double* R)
{
    const dgo_basis* B = &m->B;
    int N = B->N, n = B->n;
    for (int line = 0; line < n; ++line)
        for (int a = 0; a < N; ++a) {
            double F[4];
            fv_face_flux(m, u, gamma, e, 0, line, a, F); /* x-face (a,a+1) on row b=line */
            for (int v = 0; v < 4; ++v) {
                R[(v * n + line) * n + a] -= B->w[line] * F[v];
                R[(v * n + line) * n + a + 1] += B->w[line] * F[v];
            }
            fv_face_flux(m, u, gamma, e, 1, line, a, F); /* y-face (a,a+1) on column a'=line */
            for (int v = 0; v < 4; ++v) {
                R[(v * n + a) * n + line] -= B->w[line] * F[v];
                R[(v * n + a + 1) * n + line] += B->w[line] * F[v];
            }
        }
}

static double mass(const dgo_mesh* m, int64_t e, int a, int b)
{
    return m->hx[e] * m->hy[e] / 4.0 * m->B.w[a] * m->B.w[b];
}

static void residual(const dgo_mesh* m, const double* u, int which, double gamma, double* R)
{
    int n = m->B.n;
    int64_t ns = m->M * 3 * n * 4;
    double* HO = (double*)calloc(ns > 0 ? ns : 1, 8);
    double* LO = (double*)calloc(ns > 0 ? ns : 1, 8);
    compute_slots(m, u, gamma, HO, LO);
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < m->E; ++e) {
        double* Re = R + e * 4 * n * n;
        memset(Re, 0, sizeof(double) * 4 * n * n);
        if (which == RHS_HIGH) volume_high(m, u, gamma, e, Re);
        else volume_low(m, u, gamma, e, Re);
        add_surface(m, u, gamma, which == RHS_HIGH ? HO : LO, e, Re);
    }
    free(HO);
    free(LO);
}

int dgo_rhs(const dgo_mesh* m, const double* u, int which, double gamma, double* du)
{
    int n = m->B.n;
    residual(m, u, which, gamma, du);
    for (int64_t e = 0; e < m->E; ++e)
        for (int v = 0; v < 4; ++v)
            for (int b = 0; b < n; ++b)
                for (int a = 0; a < n; ++a) du[IDX(e, v, b, a)] /= mass(m, e, a, b);
    return 0;
}

/* ---------------------------------------------------------------------------
 * time step
 * ------------------------------------------------------------------------- */
static double lam_pair(const double* p, const double* q, int dir, double gamma)
{
    double a = dgo_wavespeed(p, dir, gamma), b = dgo_wavespeed(q, dir, gamma);
    return a > b ? a : b;
}

double dgo_max_dt(const dgo_mesh* m, const double* u, double cfl, int mode, double gamma)
{
    const dgo_basis* B = &m->B;
    int N = B->N, n = B->n;
    if (mode == DT_LOWORDER) {
        double dt = INFINITY;
        for (int64_t e = 0; e < m->E; ++e)
            for (int b = 0; b < n; ++b)
                for (int a = 0; a < n; ++a) {
                    double q[4];
                    get_node(u, n, e, a, b, q);
                    /* the low-order stability bound of eq. CFLcondition_lowordermethod
                       is only given up to a constant; the constant of the standard
                       DGSEM estimate h / ((N+1) (lambda_1 + lambda_2)) is used */
                    double t = 1.0 / ((N + 1) * (dgo_wavespeed(q, 0, gamma) / m->hx[e] +
                                                 dgo_wavespeed(q, 1, gamma) / m->hy[e]));
                    if (t < dt) dt = t;
                }
        return cfl * dt;
    }
    /* IDP: dt <= m_i / sum_j 2 d_ij, d_ij = |c_ij| lambda_ij */
    double smax = 0.0;
    double* sum = (double*)malloc(sizeof(double) * n * n);
    for (int64_t e = 0; e < m->E; ++e) {
        double hx = m->hx[e], hy = m->hy[e];
        for (int i = 0; i < n * n; ++i) sum[i] = 0.0;
        for (int line = 0; line < n; ++line)
            for (int a = 0; a < N; ++a) {
                double p[4], q[4];
                get_node(u, n, e, a, line, p);
                get_node(u, n, e, a + 1, line, q);
                double d = B->w[line] * hy / 4.0 * lam_pair(p, q, 0, gamma);
                sum[line * n + a] += 2 * d;
                sum[line * n + a + 1] += 2 * d;
                get_node(u, n, e, line, a, p);
                get_node(u, n, e, line, a + 1, q);
                d = B->w[line] * hx / 4.0 * lam_pair(p, q, 1, gamma);
                sum[a * n + line] += 2 * d;
                sum[(a + 1) * n + line] += 2 * d;
            }
        for (int f = 0; f < 4; ++f) {
            const dgo_face* F = &m->face[e * 4 + f];
            int dir = f / 2;
            for (int k = 0; k < n; ++k) {
                int a, b;
                face_node(f, k, N, &a, &b);
                double ui[4];
                get_node(u, n, e, a, b, ui);
                if (F->type == FACE_CONF || F->type == FACE_BOUNDARY) {
                    double uo[4];
                    across_node(m, u, gamma, e, f, k, ui, uo);
                    sum[b * n + a] += 2 * B->w[k] * face_len(m, e, f) / 4.0 * lam_pair(ui, uo, dir, gamma);
                } else if (F->type == FACE_LARGE) {
                    const dgo_mortar* M = &m->mort[F->mortar];
                    for (int h = 0; h < 2; ++h)
                        for (int l = 0; l < n; ++l) {
                            double wt = B->Wt[k][h * n + l];
                            if (wt == 0.0) continue;
                            int a2, b2;
                            face_node(f ^ 1, l, N, &a2, &b2);
                            double uo[4];
                            get_node(u, n, M->small[h], a2, b2, uo);
                            sum[b * n + a] += 2 * (wt * face_len(m, e, f) / 4.0) * lam_pair(ui, uo, dir, gamma);
                        }
                } else {
                    const dgo_mortar* M = &m->mort[F->mortar];
                    for (int kk = 0; kk < n; ++kk) {
                        double wt = B->Wt[kk][F->half * n + k];
                        if (wt == 0.0) continue;
                        int a2, b2;
                        face_node(M->face, kk, N, &a2, &b2);
                        double uo[4];
                        get_node(u, n, M->large, a2, b2, uo);
                        double hL = face_len(m, M->large, M->face);
                        sum[b * n + a] += 2 * (wt * hL / 4.0) * lam_pair(ui, uo, dir, gamma);
                    }
                }
            }
        }
        for (int b = 0; b < n; ++b)
            for (int a = 0; a < n; ++a) {
                double s = sum[b * n + a] / mass(m, e, a, b);
                if (s > smax) smax = s;
            }
    }
    free(sum);
    return cfl / smax;
}

/* ---------------------------------------------------------------------------
 * limiting
 * ------------------------------------------------------------------------- */

/* the limiter aims at the bounds raised by this relative margin, so that the
   rounding of the final sums cannot cross the bounds themselves */
#define BOUND_MARGIN (1.0 + 0x1p-40)
#define BOUND_MARGIN_HI (1.0 - 0x1p-40)
/* the mortar correction aims at half that margin: a node that the volume
   limiter left on its target keeps 2^-41 of room, instead of a zero or one
   mortar factor decided by the sign of a rounding error */
#define MORTAR_MARGIN (1.0 + 0x1p-41)
#define MORTAR_MARGIN_HI (1.0 - 0x1p-41)
/* local bounds hold only up to rounding for the low-order state itself (it is
   a convex combination of bar states in exact arithmetic); the bound check
   allows this relative slack for them */
#define LOCAL_TOL 1e-12
/* density increments (per node and step) this small relative to the density are
   not limited against the local density bounds */
#define LOCAL_NEGL 1e-14
/* With bounds from the low-order solution the entropy target never lies above
   the node's own low-order state: it is the smaller of the margin-raised bound
   and the node's low-order specific entropy lowered by a relative 2^-41 (volume
   step) or 2^-40 (mortar step).  Eq. Bounds_LowOrder includes the node itself
   in the neighbourhood, so where it is the minimum the raised bound would lie
   above the state the limiter starts from, and the factor would be 0 or full by
   the sign of a rounding error.  (With bar states the node's own entry is its
   input state, not u^FV: no cap.) */
#define OWN_SLACK_VOL (1.0 - 0x1p-41)
#define OWN_SLACK_MORT (1.0 - 0x1p-40)

/* largest theta in [0,1] with rho(u0 + theta dc) > 0 and p(u0 + theta dc) >= pt.
   With rho > 0, p >= pt  <=>  g(theta) = (E - pt/(gamma-1)) rho - |m|^2/2 >= 0,
   a quadratic in theta; the admissible set along the ray is [0, theta*]. */
double dgo_theta_pressure(const double* u0, const double* dc, double pt, double gamma)
{
    double e0 = u0[3] - pt / (gamma - 1.0);
    double g0 = u0[0] * e0 - 0.5 * (u0[1] * u0[1] + u0[2] * u0[2]);
    if (!(g0 > 0.0) || !(u0[0] > 0.0)) return 0.0;
    double g1 = dc[0] * e0 + u0[0] * dc[3] - (u0[1] * dc[1] + u0[2] * dc[2]);
    double g2 = dc[0] * dc[3] - 0.5 * (dc[1] * dc[1] + dc[2] * dc[2]);
    double root = INFINITY;
    if (g2 == 0.0) {
        if (g1 < 0.0) root = -g0 / g1;
    } else {
        double disc = g1 * g1 - 4.0 * g2 * g0;
        if (disc >= 0.0) {
            double sq = sqrt(disc);
            double q = -0.5 * (g1 + (g1 >= 0.0 ? sq : -sq));
            double r1 = q / g2, r2 = g0 / q;
            if (r1 > 0.0 && r1 < root) root = r1;
            if (r2 > 0.0 && r2 < root) root = r2;
        }
    }
    if (dc[0] < 0.0) {
        double rz = -u0[0] / dc[0];
        if (rz < root) root = rz;
    }
    return root < 1.0 ? root : 1.0;
}

/* ---------------------------------------------------------------------------
 * local bounds (eq. Bounds_Barstates)
 * ------------------------------------------------------------------------- */

/* Bar state of the graph edge between uL and uR, uL on the low side along dir
   (Sec. 2.2, IDP property): (u_i + u_j)/2 - c_ij . (f_j - f_i) / (2 d_ij).
   With d_ij = |c_ij| lambda_ij and c_ij parallel to the axis, c_ij / d_ij is the
   unit normal from i to j over lambda_ij, so the bar state is
   (uL + uR)/2 - (f(uR) - f(uL)) / (2 lambda), whichever end is i. */
void dgo_bar_state(const double* uL, const double* uR, int dir, double gamma, double* ub)
{
    double fL[4], fR[4];
    dgo_flux_phys(uL, dir, gamma, fL);
    dgo_flux_phys(uR, dir, gamma, fR);
    double lam = lam_pair(uL, uR, dir, gamma);
    for (int v = 0; v < 4; ++v) ub[v] = 0.5 * (uL[v] + uR[v]) - (fR[v] - fL[v]) / (2.0 * lam);
}

/* specific entropy s = p rho^-gamma; the paper's eta = s / (gamma - 1) orders
   states the same way.  0 for a state outside the admissible set. */
double dgo_spec_entropy(const double* u, double gamma)
{
    double p = dgo_pressure(u, gamma);
    if (!(u[0] > 0.0) || !(p > 0.0)) return 0.0;
    return p * pow(u[0], -gamma);
}

static void bound_add(const double* ub, double gamma, double* lo, double* hi, double* smin)
{
    if (ub[0] < *lo) *lo = ub[0];
    if (ub[0] > *hi) *hi = ub[0];
    double s = dgo_spec_entropy(ub, gamma);
    if (s < *smin) *smin = s;
}

/* own = this node, o = the other end; own_low: this node on the low side */
static void bound_edge(const double* own, const double* o, int own_low, int dir, double gamma,
                       double* lo, double* hi, double* smin)
{
    double ub[4];
    if (own_low) dgo_bar_state(own, o, dir, gamma, ub);
    else dgo_bar_state(o, own, dir, gamma, ub);
    bound_add(ub, gamma, lo, hi, smin);
}

/* Per node i: min and max of the density and min of the specific entropy over
   the bar states of i and its low-order neighbours N(i) (the node itself is the
   bar state (i, i)).  N(i): the subcell neighbours inside the element, the
   matching node across a conforming face, and across a mortar the nodes of the
   other side whose sparse weight with i is nonzero (Sec. 2.2). */
void dgo_local_bounds(const dgo_mesh* m, const double* u, double gamma, double* rlo, double* rhi,
                      double* smin)
{
    const dgo_basis* B = &m->B;
    int N = B->N, n = B->n;
    int64_t nn = n * n;
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < m->E; ++e)
        for (int b = 0; b < n; ++b)
            for (int a = 0; a < n; ++a) {
                double ui[4], uo[4];
                get_node(u, n, e, a, b, ui);
                double lo = ui[0], hi = ui[0], sm = dgo_spec_entropy(ui, gamma);
                if (a > 0) { get_node(u, n, e, a - 1, b, uo); bound_edge(ui, uo, 0, 0, gamma, &lo, &hi, &sm); }
                if (a < N) { get_node(u, n, e, a + 1, b, uo); bound_edge(ui, uo, 1, 0, gamma, &lo, &hi, &sm); }
                if (b > 0) { get_node(u, n, e, a, b - 1, uo); bound_edge(ui, uo, 0, 1, gamma, &lo, &hi, &sm); }
                if (b < N) { get_node(u, n, e, a, b + 1, uo); bound_edge(ui, uo, 1, 1, gamma, &lo, &hi, &sm); }
                for (int f = 0; f < 4; ++f) {
                    int k = -1;
                    if (f == 0 && a == 0) k = b;
                    if (f == 1 && a == N) k = b;
                    if (f == 2 && b == 0) k = a;
                    if (f == 3 && b == N) k = a;
                    if (k < 0) continue;
                    const dgo_face* F = &m->face[e * 4 + f];
                    int dir = f / 2, own_low = f & 1;
                    if (F->type == FACE_CONF || F->type == FACE_BOUNDARY) {
                        across_node(m, u, gamma, e, f, k, ui, uo);
                        bound_edge(ui, uo, own_low, dir, gamma, &lo, &hi, &sm);
                    } else if (F->type == FACE_LARGE) {
                        const dgo_mortar* M = &m->mort[F->mortar];
                        for (int h = 0; h < 2; ++h)
                            for (int l = 0; l < n; ++l) {
                                if (B->Wt[k][h * n + l] == 0.0) continue;
                                int a2, b2;
                                face_node(f ^ 1, l, N, &a2, &b2);
                                get_node(u, n, M->small[h], a2, b2, uo);
                                bound_edge(ui, uo, own_low, dir, gamma, &lo, &hi, &sm);
                            }
                    } else {
                        const dgo_mortar* M = &m->mort[F->mortar];
                        for (int kk = 0; kk < n; ++kk) {
                            if (B->Wt[kk][F->half * n + k] == 0.0) continue;
                            int a2, b2;
                            face_node(M->face, kk, N, &a2, &b2);
                            get_node(u, n, M->large, a2, b2, uo);
                            bound_edge(ui, uo, own_low, dir, gamma, &lo, &hi, &sm);
                        }
                    }
                }
                rlo[e * nn + b * n + a] = lo;
                rhi[e * nn + b * n + a] = hi;
                smin[e * nn + b * n + a] = sm;
            }
}

/* Local bounds from the low-order solution (eq. Bounds_LowOrder): per node i
   the density range over the low-order states u^FV_j of j in {i} and N(i) (the
   same neighbours as for the bar states: subcell neighbours, the matching node
   across a conforming face, the nodes with a nonzero sparse weight across a
   mortar; a boundary face adds none), and the smallest specific entropy
   p rho^-gamma among those of them with positive density and pressure. */
static void lo_add(const double* q, double gamma, double* lo, double* hi, double* sm)
{
    if (q[0] < *lo) *lo = q[0];
    if (q[0] > *hi) *hi = q[0];
    if (q[0] > 0.0 && dgo_pressure(q, gamma) > 0.0) {
        double s = dgo_spec_entropy(q, gamma);
        if (s < *sm) *sm = s;
    }
}

void dgo_lowsol_bounds(const dgo_mesh* m, const double* ufv, double gamma, double* rlo, double* rhi,
                       double* smin)
{
    const dgo_basis* B = &m->B;
    int N = B->N, n = B->n;
    int64_t nn = n * n;
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < m->E; ++e)
        for (int b = 0; b < n; ++b)
            for (int a = 0; a < n; ++a) {
                double q[4];
                double lo = INFINITY, hi = -INFINITY, sm = INFINITY;
                get_node(ufv, n, e, a, b, q);
                lo_add(q, gamma, &lo, &hi, &sm);
                if (a > 0) { get_node(ufv, n, e, a - 1, b, q); lo_add(q, gamma, &lo, &hi, &sm); }
                if (a < N) { get_node(ufv, n, e, a + 1, b, q); lo_add(q, gamma, &lo, &hi, &sm); }
                if (b > 0) { get_node(ufv, n, e, a, b - 1, q); lo_add(q, gamma, &lo, &hi, &sm); }
                if (b < N) { get_node(ufv, n, e, a, b + 1, q); lo_add(q, gamma, &lo, &hi, &sm); }
                for (int f = 0; f < 4; ++f) {
                    int k = -1;
                    if (f == 0 && a == 0) k = b;
                    if (f == 1 && a == N) k = b;
                    if (f == 2 && b == 0) k = a;
                    if (f == 3 && b == N) k = a;
                    if (k < 0) continue;
                    const dgo_face* F = &m->face[e * 4 + f];
                    int a2, b2;
                    if (F->type == FACE_CONF) {
                        face_node(f ^ 1, k, N, &a2, &b2);
                        get_node(ufv, n, F->nbr, a2, b2, q);
                        lo_add(q, gamma, &lo, &hi, &sm);
                    } else if (F->type == FACE_LARGE) {
                        const dgo_mortar* M = &m->mort[F->mortar];
                        for (int h = 0; h < 2; ++h)
                            for (int l = 0; l < n; ++l) {
                                if (B->Wt[k][h * n + l] == 0.0) continue;
                                face_node(f ^ 1, l, N, &a2, &b2);
                                get_node(ufv, n, M->small[h], a2, b2, q);
                                lo_add(q, gamma, &lo, &hi, &sm);
                            }
                    } else if (F->type == FACE_SMALL) {
                        const dgo_mortar* M = &m->mort[F->mortar];
                        for (int kk = 0; kk < n; ++kk) {
                            if (B->Wt[kk][F->half * n + k] == 0.0) continue;
                            face_node(M->face, kk, N, &a2, &b2);
                            get_node(ufv, n, M->large, a2, b2, q);
                            lo_add(q, gamma, &lo, &hi, &sm);
                        }
                    }
                }
                rlo[e * nn + b * n + a] = lo;
                rhi[e * nn + b * n + a] = hi;
                smin[e * nn + b * n + a] = sm;
            }
}

/* psi(theta) = p(u0 + theta dc) - st rho(u0 + theta dc)^gamma and its derivative.
   psi >= 0 with rho > 0 is s >= st; psi is concave along the ray (p is concave
   in the conserved variables and rho^gamma convex). */
static double psi_entropy(const double* u0, const double* dc, double th, double st, double gamma,
                          double* dpsi)
{
    double q[4];
    for (int v = 0; v < 4; ++v) q[v] = u0[v] + th * dc[v];
    if (!(q[0] > 0.0)) {
        *dpsi = 0.0;
        return -INFINITY;
    }
    double v1 = q[1] / q[0], v2 = q[2] / q[0];
    double p = (gamma - 1.0) * (q[3] - 0.5 * (q[1] * v1 + q[2] * v2));
    double rg = st * pow(q[0], gamma);
    double dp = (gamma - 1.0) * (dc[3] - v1 * dc[1] - v2 * dc[2] + 0.5 * (v1 * v1 + v2 * v2) * dc[0]);
    *dpsi = dp - gamma * rg / q[0] * dc[0];
    return p - rg;
}

/* Largest theta in [0, thi] with s(u0 + theta dc) >= st, for a ray on which
   rho stays positive.  The admissible set of a concave psi with psi(0) >= 0 is
   an interval [0, theta*]; the root is bracketed from both sides: the chord
   through a feasible and an infeasible point cuts the axis at or below theta*
   (concavity), the Newton step from the infeasible end at or above it (the
   tangent lies above psi).  This is the two-sided iteration used for convex
   limiting by Guermond, Nazarov, Popov and Tomas (SIAM J. Sci. Comput. 2018).
   When the two estimates are within 1e-14 of each other (or cross by rounding)
   it returns the chord point, theta* up to rounding; otherwise it stops when
   the bracket is that narrow, at most 16 rounds, and returns the feasible end;
   psi(0) <= 0 returns 0. */
double dgo_theta_entropy(const double* u0, const double* dc, double st, double gamma, double thi)
{
    if (!(thi > 0.0)) return 0.0;
    double dh, dl, dx;
    double ph = psi_entropy(u0, dc, thi, st, gamma, &dh);
    if (ph >= 0.0) return thi;
    double pl = psi_entropy(u0, dc, 0.0, st, gamma, &dl);
    if (!(pl > 0.0)) return 0.0;
    double lo = 0.0, hi = thi;
    for (int it = 0; it < 16; ++it) {
        double c = lo + pl * (hi - lo) / (pl - ph);
        double nw = dh < 0.0 ? hi - ph / dh : hi;
        if (!(c > lo)) c = lo;
        if (!(c < hi)) c = hi;
        if (!(nw < hi)) nw = hi;
        if (nw < c) nw = c;
        double pc = psi_entropy(u0, dc, c, st, gamma, &dx);
        if (pc >= 0.0) {
            lo = c;
            pl = pc;
        } else {
            hi = c;
            ph = pc;
            dh = dx;
        }
        // the estimates meet: c is theta* up to rounding
        if (nw - c <= 1e-14) return c;
        double pn = psi_entropy(u0, dc, nw, st, gamma, &dx);
        if (pn >= 0.0) {
            if (nw > lo) {
                lo = nw;
                pl = pn;
            }
        } else if (nw < hi) {
            hi = nw;
            ph = pn;
            dh = dx;
        }
        if (hi - lo <= 1e-14) break;
    }
    return lo;
}

/* ---------------------------------------------------------------------------
 * shock indicator for combined limiting (Sec. 3.5, eq. combination_posLim_local)
 * ------------------------------------------------------------------------- */

/* Per element: the Hennemann indicator on the pressure.  The nodal pressure is
   expanded in orthonormal Legendre modes m_ij (the inverse of interpolation at
   the LGL nodes); energy = max of the energy fractions of the highest mode
   shell and of the second-highest shell within the modes up to N-1; alpha =
   1 / (1 + exp(-(s/T)(energy - T))), T = 0.5 10^(-1.8 (N+1)^(1/4)),
   s = ln(9999); values below 1e-3 become 0.  Not capped: alpha in [0, 1]. */
void dgo_shock_indicator(const dgo_mesh* m, const double* u, double gamma, double* ind)
{
    const dgo_basis* B = &m->B;
    int N = B->N, n = B->n;
    /* V[a][i] = sqrt((2i+1)/2) L_i(xi_a); Vi = V^-1 by Gauss-Jordan elimination */
    double V[DGO_NMAX][2 * DGO_NMAX], Vi[DGO_NMAX][DGO_NMAX];
    for (int a = 0; a < n; ++a)
        for (int i = 0; i < 2 * n; ++i)
            V[a][i] = i < n ? sqrt((2.0 * i + 1.0) / 2.0) * dgo_legendre(i, B->xi[a]) : (i - n == a ? 1.0 : 0.0);
    for (int c = 0; c < n; ++c) {
        int piv = c;
        for (int r = c + 1; r < n; ++r)
            if (fabs(V[r][c]) > fabs(V[piv][c])) piv = r;
        for (int k = 0; k < 2 * n; ++k) {
            double t = V[c][k];
            V[c][k] = V[piv][k];
            V[piv][k] = t;
        }
        double d = V[c][c];
        for (int k = 0; k < 2 * n; ++k) V[c][k] /= d;
        for (int r = 0; r < n; ++r) {
            if (r == c) continue;
            double f = V[r][c];
            for (int k = 0; k < 2 * n; ++k) V[r][k] -= f * V[c][k];
        }
    }
    for (int i = 0; i < n; ++i)
        for (int a = 0; a < n; ++a) Vi[i][a] = V[i][n + a];
    double T = 0.5 * pow(10.0, -1.8 * pow(N + 1.0, 0.25));
    double sharp = log((1.0 - 1e-4) / 1e-4);
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < m->E; ++e) {
        double pq[DGO_NMAX][DGO_NMAX]; /* [b][a] */
        for (int b = 0; b < n; ++b)
            for (int a = 0; a < n; ++a) {
                double q[4];
                get_node(u, n, e, a, b, q);
                pq[b][a] = dgo_pressure(q, gamma);
            }
        double all = 0.0, low1 = 0.0, low2 = 0.0;
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                double mij = 0.0;
                for (int b = 0; b < n; ++b)
                    for (int a = 0; a < n; ++a) mij += Vi[i][a] * Vi[j][b] * pq[b][a];
                double m2 = mij * mij;
                all += m2;
                if (i < N && j < N) low1 += m2;
                if (i < N - 1 && j < N - 1) low2 += m2;
            }
        double en1 = (all - low1) / all, en2 = (low1 - low2) / low1;
        double en = en1 > en2 ? en1 : en2;
        double al = 1.0 / (1.0 + exp(-(sharp / T) * (en - T)));
        ind[e] = al < 1e-3 ? 0.0 : al;
    }
}

/* Node factor of the volume limiter from the node's face increments cf (nf of
   them, dt/m_i-scaled): Zalesak factors for the density floor (and, with loc,
   the ceiling), the pressure root per face and, with loc, the entropy root per
   face, the last two on Gamma = 4-scaled increments. */
static double volume_node_factor(const double* q, double cf[4][4], int nf, double rfloor, double pfloor,
                                 int loc, double rceil, double sm, int cap, double gamma)
{
    /* (q is the node's low-order state u^FV; cap: entropy target capped by it) */
    double rt = rfloor * BOUND_MARGIN, pt = pfloor * BOUND_MARGIN;
    /* Zalesak: the sum of the negative (positive) density increments may use
       at most the distance to the lower (upper) bound */
    double P = 0.0, Pp = 0.0;
    for (int j = 0; j < nf; ++j) {
        if (cf[j][0] < 0.0) P += cf[j][0];
        if (cf[j][0] > 0.0) Pp += cf[j][0];
    }
    double t = 1.0;
    /* local bounds: increments below 1e-14 of the density are rounding noise
       and are not limited (a node whose density interval has zero width would
       otherwise switch between theta = 0 and 1 on the sign of a rounding error) */
    if (loc && P > -LOCAL_NEGL * q[0]) P = 0.0;
    if (loc && Pp < LOCAL_NEGL * q[0]) Pp = 0.0;
    if (P < 0.0) {
        double r = (rt - q[0]) / P;
        t = r < 1.0 ? r : 1.0;
        if (t < 0.0) t = 0.0;
    }
    if (loc && Pp > 0.0) {
        double r = (rceil * BOUND_MARGIN_HI - q[0]) / Pp;
        if (r < 0.0) r = 0.0;
        if (r < t) t = r;
    }
    for (int j = 0; j < nf; ++j) {
        double dc[4];
        for (int v = 0; v < 4; ++v) dc[v] = 4.0 * cf[j][v];
        double tp = dgo_theta_pressure(q, dc, pt, gamma);
        if (tp < t) t = tp;
    }
    /* entropy: per face on [0, t], target capped by the node's own entropy */
    if (loc) {
        double st = sm * BOUND_MARGIN;
        const double own = dgo_spec_entropy(q, gamma) * OWN_SLACK_VOL;
        if (cap && own < st) st = own;
        for (int j = 0; j < nf; ++j) {
            double dc[4];
            for (int v = 0; v < 4; ++v) dc[v] = 4.0 * cf[j][v];
            t = dgo_theta_entropy(q, dc, st, gamma, t);
        }
    }
    return t;
}

/* Factor of one mortar node with its n_i-scaled increment dc: density floor
   (and ceiling), pressure root, entropy root, against half the volume margin;
   q is u^vol, sfv the specific entropy of the node's low-order state (the cap
   of the entropy target). */
static double mortar_node_factor(const double* q, const double* dc, double rfloor, double pfloor, int loc,
                                 double rceil, double sm, double sfv, double gamma)
{
    double rt = rfloor * MORTAR_MARGIN, pt = pfloor * MORTAR_MARGIN;
    double tn = 1.0;
    const int negl = loc && fabs(dc[0]) <= LOCAL_NEGL * q[0];
    if (dc[0] < 0.0 && !negl) {
        double r = (rt - q[0]) / dc[0];
        if (r < 0.0) r = 0.0;
        if (r < tn) tn = r;
    }
    if (loc && dc[0] > 0.0 && !negl) {
        double r = (rceil * MORTAR_MARGIN_HI - q[0]) / dc[0];
        if (r < 0.0) r = 0.0;
        if (r < tn) tn = r;
    }
    double tp = dgo_theta_pressure(q, dc, pt, gamma);
    if (tp < tn) tn = tp;
    if (loc) {
        double st = sm * MORTAR_MARGIN;
        if (sfv * OWN_SLACK_MORT < st) st = sfv * OWN_SLACK_MORT;
        tn = dgo_theta_entropy(q, dc, st, gamma, tn);
    }
    return tn;
}

int dgo_fe_step(const dgo_mesh* m, const double* u, double dt, double gamma, double beta,
                int limiter, double* out, dgo_stats* st)
{
    return dgo_fe_step_ind(m, u, dt, gamma, beta, limiter, 0, out, st);
}

int dgo_fe_step_ind(const dgo_mesh* m, const double* u, double dt, double gamma, double beta,
                    int limiter, const double* ind_in, double* out, dgo_stats* st)
{
    return dgo_fe_step_detail(m, u, dt, gamma, beta, limiter, ind_in, out, st, 0, 0, 0);
}

int dgo_fe_step_detail(const dgo_mesh* m, const double* u, double dt, double gamma, double beta,
                       int limiter, const double* ind_in, double* out, dgo_stats* st, double* uvol_out,
                       double* dslot_out, double* theta_out)
{
    const dgo_basis* B = &m->B;
    int N = B->N, n = B->n;
    int64_t E = m->E, nn = n * n;
    memset(st, 0, sizeof(*st));
    st->dt = dt;
    st->theta_vol_min = 1.0;
    st->theta_mort_min = 1.0;
    int64_t ns = m->M * 3 * n * 4;
    double* HO = (double*)calloc(ns > 0 ? ns : 1, 8);
    double* LO = (double*)calloc(ns > 0 ? ns : 1, 8);
    compute_slots(m, u, gamma, HO, LO);
    if (dslot_out)
        for (int64_t i = 0; i < ns; ++i) dslot_out[i] = HO[i] - LO[i];

    if (limiter == LIM_NONE) {
        double* R = (double*)malloc(sizeof(double) * E * 4 * nn);
        residual(m, u, RHS_HIGH, gamma, R);
        for (int64_t e = 0; e < E; ++e)
            for (int v = 0; v < 4; ++v)
                for (int b = 0; b < n; ++b)
                    for (int a = 0; a < n; ++a)
                        out[IDX(e, v, b, a)] = u[IDX(e, v, b, a)] + dt / mass(m, e, a, b) * R[IDX(e, v, b, a)];
        free(R);
        free(HO);
        free(LO);
        return 0;
    }

    double* uFV = (double*)malloc(sizeof(double) * E * 4 * nn);
    double* rmin = (double*)malloc(sizeof(double) * E * nn);
    double* pmin = (double*)malloc(sizeof(double) * E * nn);
    /* local: local bounds enforced; comb: positivity and local factors both
       computed and blended per element with the shock indicator */
    const int comb = limiter == LIM_COMBINED;
    const int pure_local = limiter == LIM_LOCAL || limiter == LIM_LOCAL_LO;
    const int local = pure_local || comb;
    const int cap_own = limiter == LIM_LOCAL_LO;
    double *rlo = 0, *rhi = 0, *smin = 0, *ind = 0;
    if (local) {
        rlo = (double*)malloc(sizeof(double) * E * nn);
        rhi = (double*)malloc(sizeof(double) * E * nn);
        smin = (double*)malloc(sizeof(double) * E * nn);
        if (limiter == LIM_LOCAL_LO) {
            /* the low-order solution first (the same arithmetic as below), then
               its bounds */
#pragma omp parallel for schedule(static)
            for (int64_t e = 0; e < E; ++e) {
                double R[4 * DGO_NMAX * DGO_NMAX];
                memset(R, 0, sizeof(R));
                volume_low(m, u, gamma, e, R);
                add_surface(m, u, gamma, LO, e, R);
                for (int v = 0; v < 4; ++v)
                    for (int b = 0; b < n; ++b)
                        for (int a = 0; a < n; ++a)
                            uFV[IDX(e, v, b, a)] =
                                u[IDX(e, v, b, a)] + dt / mass(m, e, a, b) * R[(v * n + b) * n + a];
            }
            dgo_lowsol_bounds(m, uFV, gamma, rlo, rhi, smin);
        } else {
            dgo_local_bounds(m, u, gamma, rlo, rhi, smin);
        }
    }
    if (comb) {
        ind = (double*)malloc(sizeof(double) * (E > 0 ? E : 1));
        if (ind_in) memcpy(ind, ind_in, sizeof(double) * E);
        else dgo_shock_indicator(m, u, gamma, ind);
    }
    int64_t nfaces = 0;
    double alpha_sum = 0.0;
    int64_t inadm = 0, viol = 0;
    double thmin = 1.0;

#pragma omp parallel for schedule(static) reduction(+ : nfaces, alpha_sum, inadm) reduction(min : thmin)
    for (int64_t e = 0; e < E; ++e) {
        double R[4 * DGO_NMAX * DGO_NMAX];
        memset(R, 0, sizeof(R));
        volume_low(m, u, gamma, e, R);
        add_surface(m, u, gamma, LO, e, R);
        /* low-order update and bounds (eq. Bounds_Positivity) */
        for (int b = 0; b < n; ++b)
            for (int a = 0; a < n; ++a) {
                double q[4];
                for (int v = 0; v < 4; ++v) {
                    q[v] = u[IDX(e, v, b, a)] + dt / mass(m, e, a, b) * R[(v * n + b) * n + a];
                    uFV[IDX(e, v, b, a)] = q[v];
                }
                double p = dgo_pressure(q, gamma);
                if (!(q[0] > 0.0) || !(p > 0.0)) inadm++;
                rmin[e * nn + b * n + a] = beta * q[0];
                pmin[e * nn + b * n + a] = beta * p;
                /* local limiting keeps the positivity bounds as well: its
                   density floor is the larger of the two */
                if (local && rlo[e * nn + b * n + a] < rmin[e * nn + b * n + a])
                    rlo[e * nn + b * n + a] = rmin[e * nn + b * n + a];
            }
        /* antidiffusive fluxes on interior subcell faces: telescoped high-order
           flux (eq. fluxdifferencingform) minus the low-order subcell flux */
        double Ax[DGO_NMAX][DGO_NMAX][4], Ay[DGO_NMAX][DGO_NMAX][4]; /* [line][a] */
        for (int line = 0; line < n; ++line)
            for (int a = 0; a < N; ++a) {
                for (int dir = 0; dir < 2; ++dir) {
                    double fho[4] = {0, 0, 0, 0}, ffv[4];
                    double s = (dir == 0 ? m->hy[e] : m->hx[e]) / 2.0;
                    for (int l = 0; l <= a; ++l)
                        for (int k = 0; k < n; ++k) {
                            double ul[4], uk[4], fs[4];
                            if (dir == 0) {
                                get_node(u, n, e, l, line, ul);
                                get_node(u, n, e, k, line, uk);
                            } else {
                                get_node(u, n, e, line, l, ul);
                                get_node(u, n, e, line, k, uk);
                            }
                            dgo_flux_volume(m->vflux, ul, uk, dir, gamma, fs);
                            for (int v = 0; v < 4; ++v) fho[v] += B->S[l][k] * s * fs[v];
                        }
                    fv_face_flux(m, u, gamma, e, dir, line, a, ffv);
                    for (int v = 0; v < 4; ++v) {
                        double A = B->w[line] * (fho[v] - ffv[v]);
                        if (dir == 0) Ax[line][a][v] = A;
                        else Ay[line][a][v] = A;
                    }
                }
            }
        /* per-node factors (positivity, local, or both for the blend) */
        double th[DGO_NMAX][DGO_NMAX], thl[DGO_NMAX][DGO_NMAX]; /* [b][a] */
        for (int b = 0; b < n; ++b)
            for (int a = 0; a < n; ++a) {
                double mi = mass(m, e, a, b);
                double q[4];
                for (int v = 0; v < 4; ++v) q[v] = uFV[IDX(e, v, b, a)];
                double cf[4][4];
                int nf = 0;
                if (a > 0) { for (int v = 0; v < 4; ++v) cf[nf][v] = dt / mi * Ax[b][a - 1][v]; nf++; }
                if (a < N) { for (int v = 0; v < 4; ++v) cf[nf][v] = -dt / mi * Ax[b][a][v]; nf++; }
                if (b > 0) { for (int v = 0; v < 4; ++v) cf[nf][v] = dt / mi * Ay[a][b - 1][v]; nf++; }
                if (b < N) { for (int v = 0; v < 4; ++v) cf[nf][v] = -dt / mi * Ay[a][b][v]; nf++; }
                int64_t i = e * nn + b * n + a;
                if (pure_local) {
                    th[b][a] = volume_node_factor(q, cf, nf, rlo[i], pmin[i], 1, rhi[i], smin[i], cap_own, gamma);
                } else {
                    th[b][a] = volume_node_factor(q, cf, nf, rmin[i], pmin[i], 0, 0.0, 0.0, 0, gamma);
                    if (comb)
                        thl[b][a] = volume_node_factor(q, cf, nf, rlo[i], pmin[i], 1, rhi[i], smin[i], cap_own, gamma);
                }
            }
        /* face factor: the smaller node factor of its two nodes, combined:
           (1 - w) theta_pos + w theta_local with the element's indicator w */
        const double w = comb ? ind[e] : 0.0;
#define FACE_T(b1, a1, b2, a2)                                                                 \
    (comb ? (1.0 - w) * (th[b1][a1] < th[b2][a2] ? th[b1][a1] : th[b2][a2]) +                 \
                w * (thl[b1][a1] < thl[b2][a2] ? thl[b1][a1] : thl[b2][a2])                   \
          : (th[b1][a1] < th[b2][a2] ? th[b1][a1] : th[b2][a2]))
        /* per-face factor = min of its two nodes; limited volume update */
        for (int b = 0; b < n; ++b)
            for (int a = 0; a < n; ++a) {
                double mi = mass(m, e, a, b);
                double acc[4];
                for (int v = 0; v < 4; ++v) acc[v] = uFV[IDX(e, v, b, a)];
                if (a > 0) {
                    double t = FACE_T(b, a - 1, b, a);
                    for (int v = 0; v < 4; ++v) acc[v] += t * dt / mi * Ax[b][a - 1][v];
                }
                if (a < N) {
                    double t = FACE_T(b, a, b, a + 1);
                    for (int v = 0; v < 4; ++v) acc[v] -= t * dt / mi * Ax[b][a][v];
                    nfaces++;
                    alpha_sum += 1.0 - t;
                    if (t < thmin) thmin = t;
                }
                if (b > 0) {
                    double t = FACE_T(b - 1, a, b, a);
                    for (int v = 0; v < 4; ++v) acc[v] += t * dt / mi * Ay[a][b - 1][v];
                }
                if (b < N) {
                    double t = FACE_T(b, a, b + 1, a);
                    for (int v = 0; v < 4; ++v) acc[v] -= t * dt / mi * Ay[a][b][v];
                    nfaces++;
                    alpha_sum += 1.0 - t;
                    if (t < thmin) thmin = t;
                }
                for (int v = 0; v < 4; ++v) out[IDX(e, v, b, a)] = acc[v];
            }
#undef FACE_T
    }
    st->fv_inadmissible = inadm;
    st->theta_vol_min = thmin;
    st->alpha_vol_mean = nfaces ? alpha_sum / nfaces : 0.0;
    if (uvol_out) memcpy(uvol_out, out, sizeof(double) * E * 4 * nn);

    /* mortar correction: one factor per mortar, antidiffusive flux scaled by
       the number n_i of mortars at node i (Sec. 2.3, remark on mortar limiting) */
    if (m->M > 0) {
        double* theta = (double*)malloc(sizeof(double) * m->M);
        double tmsum = 0.0, tmmin = 1.0;
#pragma omp parallel for schedule(static) reduction(+ : tmsum) reduction(min : tmmin)
        for (int64_t S = 0; S < m->M; ++S) {
            const dgo_mortar* M = &m->mort[S];
            double t = 1.0, tl = 1.0; /* positivity (or local) factor; local factor of the blend */
            for (int s = 0; s < 3 * n; ++s) {
                int64_t e;
                int f, k;
                if (s < n) { e = M->large; f = M->face; k = s; }
                else { int h = (s - n) / n; e = M->small[h]; f = M->face ^ 1; k = (s - n) % n; }
                int a, b;
                face_node(f, k, N, &a, &b);
                int ni = 0;
                if (a == 0 && is_mortar(m->face[e * 4 + 0].type)) ni++;
                if (a == N && is_mortar(m->face[e * 4 + 1].type)) ni++;
                if (b == 0 && is_mortar(m->face[e * 4 + 2].type)) ni++;
                if (b == N && is_mortar(m->face[e * 4 + 3].type)) ni++;
                double mi = mass(m, e, a, b);
                double q[4], dc[4];
                const double* ho = HO + (S * 3 * n + s) * 4;
                const double* lo = LO + (S * 3 * n + s) * 4;
                for (int v = 0; v < 4; ++v) {
                    q[v] = out[IDX(e, v, b, a)];
                    dc[v] = ni * dt / mi * (ho[v] - lo[v]);
                }
                /* the high-order mortar flux interpolates the large face; near
                   vacuum that state can leave the admissible set and the flux is
                   not defined: the mortar then keeps the low-order flux (Sec. 3.2) */
                if (!(isfinite(dc[0]) && isfinite(dc[1]) && isfinite(dc[2]) && isfinite(dc[3]))) {
                    t = tl = 0.0;
                    continue;
                }
                /* this node's factor, then the minimum over the mortar's nodes */
                int64_t i = e * nn + b * n + a;
                double sfv = INFINITY;
                if (cap_own) {
                    double qf[4];
                    get_node(uFV, n, e, a, b, qf);
                    sfv = dgo_spec_entropy(qf, gamma);
                }
                double tn = pure_local
                                ? mortar_node_factor(q, dc, rlo[i], pmin[i], 1, rhi[i], smin[i], sfv, gamma)
                                : mortar_node_factor(q, dc, rmin[i], pmin[i], 0, 0.0, 0.0, 0.0, gamma);
                if (tn < t) t = tn;
                if (comb) {
                    double tnl = mortar_node_factor(q, dc, rlo[i], pmin[i], 1, rhi[i], smin[i], sfv, gamma);
                    if (tnl < tl) tl = tnl;
                }
            }
            /* combined: the mortar's weight is the largest indicator of its
               three elements */
            if (comb) {
                double w = ind[M->large];
                if (ind[M->small[0]] > w) w = ind[M->small[0]];
                if (ind[M->small[1]] > w) w = ind[M->small[1]];
                t = (1.0 - w) * t + w * tl;
            }
            theta[S] = t;
            tmsum += 1.0 - t;
            if (t < tmmin) tmmin = t;
        }
        st->alpha_mort_mean = tmsum / m->M;
        st->theta_mort_min = tmmin;
        if (theta_out) memcpy(theta_out, theta, sizeof(double) * m->M);
        /* apply: each node gathers its mortars in ascending mortar id */
#pragma omp parallel for schedule(static)
        for (int64_t e = 0; e < E; ++e) {
            for (int b = 0; b < n; ++b)
                for (int a = 0; a < n; ++a) {
                    int64_t slots[2];
                    int64_t ids[2];
                    int cnt = 0;
                    for (int f = 0; f < 4; ++f) {
                        int k = -1;
                        if (f == 0 && a == 0) k = b;
                        if (f == 1 && a == N) k = b;
                        if (f == 2 && b == 0) k = a;
                        if (f == 3 && b == N) k = a;
                        if (k < 0) continue;
                        int64_t s = face_slot(m, e, f, k);
                        if (s < 0) continue;
                        slots[cnt] = s;
                        ids[cnt] = m->face[e * 4 + f].mortar;
                        cnt++;
                    }
                    if (cnt == 2 && ids[1] < ids[0]) {
                        int64_t t = slots[0]; slots[0] = slots[1]; slots[1] = t;
                        t = ids[0]; ids[0] = ids[1]; ids[1] = t;
                    }
                    double mi = mass(m, e, a, b);
                    for (int c = 0; c < cnt; ++c) {
                        const double* ho = HO + slots[c] * 4;
                        const double* lo = LO + slots[c] * 4;
                        double t = theta[ids[c]];
                        if (t == 0.0) continue;
                        for (int v = 0; v < 4; ++v) out[IDX(e, v, b, a)] += t * dt / mi * (ho[v] - lo[v]);
                    }
                }
        }
        free(theta);
    }
    /* bound check of the final state against the bounds themselves */
#pragma omp parallel for schedule(static) reduction(+ : viol)
    for (int64_t e = 0; e < E; ++e)
        for (int b = 0; b < n; ++b)
            for (int a = 0; a < n; ++a) {
                double q[4];
                get_node(out, n, e, a, b, q);
                int64_t i = e * nn + b * n + a;
                /* combined limiting guarantees the positivity bounds only */
                if (!pure_local) {
                    if (q[0] < rmin[i] || dgo_pressure(q, gamma) < pmin[i] || q[0] != q[0]) viol++;
                } else if (!(q[0] >= rlo[i] * (1.0 - LOCAL_TOL)) || q[0] > rhi[i] * (1.0 + LOCAL_TOL) ||
                           dgo_pressure(q, gamma) < pmin[i] ||
                           dgo_spec_entropy(q, gamma) < smin[i] * (1.0 - LOCAL_TOL)) {
                    viol++;
                }
            }
    st->violations = viol;
    free(uFV);
    free(rmin);
    free(pmin);
    free(rlo);
    free(rhi);
    free(smin);
    free(ind);
    free(HO);
    free(LO);
    return st->fv_inadmissible ? 1 : 0;
}

int dgo_ssprk3(const dgo_mesh* m, double* u, double cfl, int mode, double gamma, double beta,
               int limiter, dgo_stats* st)
{
    return dgo_ssprk3_dt(m, u, dgo_max_dt(m, u, cfl, mode, gamma), gamma, beta, limiter, st);
}

int dgo_ssprk3_dt(const dgo_mesh* m, double* u, double dt, double gamma, double beta, int limiter,
                  dgo_stats* st)
{
    int n = m->B.n;
    int64_t sz = m->E * 4 * n * n;
    double* u1 = (double*)malloc(sizeof(double) * sz);
    double* w = (double*)malloc(sizeof(double) * sz);
    dgo_stats s1, s2, s3;
    int rc = 0;
    rc |= dgo_fe_step(m, u, dt, gamma, beta, limiter, u1, &s1);
    rc |= dgo_fe_step(m, u1, dt, gamma, beta, limiter, w, &s2);
    for (int64_t i = 0; i < sz; ++i) u1[i] = 0.75 * u[i] + 0.25 * w[i];
    rc |= dgo_fe_step(m, u1, dt, gamma, beta, limiter, w, &s3);
    for (int64_t i = 0; i < sz; ++i) u[i] = u[i] / 3.0 + 2.0 / 3.0 * w[i];
    memset(st, 0, sizeof(*st));
    st->dt = dt;
    st->fv_inadmissible = s1.fv_inadmissible + s2.fv_inadmissible + s3.fv_inadmissible;
    st->violations = s1.violations + s2.violations + s3.violations;
    st->theta_vol_min = fmin(s1.theta_vol_min, fmin(s2.theta_vol_min, s3.theta_vol_min));
    st->theta_mort_min = fmin(s1.theta_mort_min, fmin(s2.theta_mort_min, s3.theta_mort_min));
    st->alpha_vol_mean = (s1.alpha_vol_mean + s2.alpha_vol_mean + s3.alpha_vol_mean) / 3.0;
    st->alpha_mort_mean = (s1.alpha_mort_mean + s2.alpha_mort_mean + s3.alpha_mort_mean) / 3.0;
    free(u1);
    free(w);
    return rc;
}
