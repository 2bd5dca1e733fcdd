/*
 * Oracle: one-dimensional LGL basis, SBP operators, mortar interpolation and
 * L2 projection, and the sparsified mortar weights.
 * TEST INFRASTRUCTURE ONLY (see dgo.h).
 *
 *  - LGL nodes/weights, Lagrange basis, omega_i = integral of phi_i: Sec. 2.1.
 *  - Qbar_ij = omega_i phi_j'(xi_i), Bbar = diag(-1,0,..,0,1), Sbar = 2 Qbar - Bbar:
 *    Sec. 2.1, volume-integral term of eq. (evolutionformula).
 *  - Interpolation of the large face to the two mortars and the L2 projection
 *    back (Kopriva's mortar, cited in Sec. 2.2 and Sec. 2.3).
 *  - Sparse weights tilde-omega = overlap length of the LGL subcells:
 *    eq. (local_weights), App. A.
 */
#include <math.h>
#include <string.h>

#include "dgo.h"

/* Legendre polynomial L_m(s) by the three-term recurrence (long double). */
static long double leg(int m, long double s, long double* dleg)
{
    long double p0 = 1.0L, p1 = s, d0 = 0.0L, d1 = 1.0L;
    if (m == 0) {
        if (dleg) *dleg = 0.0L;
        return 1.0L;
    }
    for (int k = 2; k <= m; ++k) {
        long double p2 = ((2 * k - 1) * s * p1 - (k - 1) * p0) / k;
        long double d2 = d0 + (2 * k - 1) * p1; /* L_k' = L_{k-2}' + (2k-1) L_{k-1} */
        p0 = p1;
        p1 = p2;
        d0 = d1;
        d1 = d2;
    }
    if (dleg) *dleg = d1;
    return p1;
}

double dgo_legendre(int m, double s) { return (double)leg(m, s, 0); }

/* Second derivative of L_N from the Legendre ODE: (1-s^2) L'' = 2 s L' - N(N+1) L. */
static void lgl_nodes(int N, long double* x, long double* w)
{
    x[0] = -1.0L;
    x[N] = 1.0L;
    for (int j = 1; j < N; ++j) {
        /* interior nodes: roots of L_N', Newton from Chebyshev-Lobatto guesses */
        long double s = -cosl(3.14159265358979323846264338327950288L * j / N);
        for (int it = 0; it < 100; ++it) {
            long double d;
            long double l = leg(N, s, &d);
            long double dd = (2.0L * s * d - N * (N + 1) * l) / (1.0L - s * s);
            long double ds = d / dd;
            s -= ds;
            if (fabsl(ds) < 1e-30L) break;
        }
        x[j] = s;
    }
    for (int j = 0; j <= N; ++j) {
        long double l = leg(N, x[j], 0);
        w[j] = 2.0L / (N * (N + 1) * l * l);
    }
}

/* Gauss-Legendre: roots of L_q, weights 2 / ((1-s^2) L_q'(s)^2). */
static void gauss_nodes(int q, long double* x, long double* w)
{
    for (int j = 0; j < q; ++j) {
        long double s = -cosl(3.14159265358979323846264338327950288L * (j + 0.75L) / (q + 0.5L));
        for (int it = 0; it < 100; ++it) {
            long double d;
            long double l = leg(q, s, &d);
            long double ds = l / d;
            s -= ds;
            if (fabsl(ds) < 1e-30L) break;
        }
        long double d;
        leg(q, s, &d);
        x[j] = s;
        w[j] = 2.0L / ((1.0L - s * s) * d * d);
    }
}

static long double lagr(int n, const long double* xi, int k, long double s)
{
    long double r = 1.0L;
    for (int m = 0; m < n; ++m)
        if (m != k) r *= (s - xi[m]) / (xi[k] - xi[m]);
    return r;
}

double dgo_lagrange(const dgo_basis* B, int k, double s)
{
    long double xi[DGO_NMAX];
    for (int i = 0; i < B->n; ++i) xi[i] = B->xi[i];
    return (double)lagr(B->n, xi, k, s);
}

int dgo_basis_init(dgo_basis* B, int N)
{
    if (N < 1 || N + 1 > DGO_NMAX) return -1;
    memset(B, 0, sizeof(*B));
    int n = N + 1;
    B->N = N;
    B->n = n;
    long double x[DGO_NMAX], w[DGO_NMAX];
    lgl_nodes(N, x, w);
    for (int i = 0; i < n; ++i) {
        B->xi[i] = (double)x[i];
        B->w[i] = (double)w[i];
    }

    /* D[a][k] = phi_k'(xi_a), barycentric form */
    long double bw[DGO_NMAX], Dl[DGO_NMAX][DGO_NMAX];
    for (int j = 0; j < n; ++j) {
        long double p = 1.0L;
        for (int k = 0; k < n; ++k)
            if (k != j) p *= (x[j] - x[k]);
        bw[j] = 1.0L / p;
    }
    for (int a = 0; a < n; ++a) {
        long double diag = 0.0L;
        for (int k = 0; k < n; ++k) {
            if (k == a) continue;
            Dl[a][k] = (bw[k] / bw[a]) / (x[a] - x[k]);
            diag -= Dl[a][k];
        }
        Dl[a][a] = diag;
    }
    /* Sbar = 2 diag(w) D - Bbar */
    for (int a = 0; a < n; ++a)
        for (int k = 0; k < n; ++k) {
            B->D[a][k] = (double)Dl[a][k];
            long double s = 2.0L * w[a] * Dl[a][k];
            if (a == k && a == 0) s += 1.0L;
            if (a == k && a == N) s -= 1.0L;
            B->S[a][k] = (double)s;
        }

    /* interpolation to the lower (h=0) / upper (h=1) half: s = (xi_l -/+ 1)/2 */
    for (int h = 0; h < 2; ++h) {
        long double sh = h == 0 ? -1.0L : 1.0L;
        for (int l = 0; l < n; ++l)
            for (int k = 0; k < n; ++k) B->I[h][l][k] = (double)lagr(n, x, k, (x[l] + sh) / 2.0L);
    }

    /* exact L2 projection of a per-half degree-N polynomial onto degree N on
       [-1,1], modal: c_m = (2m+1)/2 * integral(g L_m); each half integral by
       (N+1)-point Gauss-Legendre, exact for degree 2N. */
    {
        long double gx[DGO_NMAX + 1], gw[DGO_NMAX + 1];
        int q = n;
        gauss_nodes(q, gx, gw);
        for (int h = 0; h < 2; ++h) {
            long double sh = h == 0 ? -1.0L : 1.0L;
            for (int k = 0; k < n; ++k)
                for (int l = 0; l < n; ++l) {
                    long double acc = 0.0L;
                    for (int m = 0; m <= N; ++m) {
                        long double integ = 0.0L;
                        for (int j = 0; j < q; ++j)
                            integ += gw[j] * lagr(n, x, l, gx[j]) * leg(m, (gx[j] + sh) / 2.0L, 0);
                        integ *= 0.5L; /* ds = dt/2 on a half */
                        acc += leg(m, x[k], 0) * (2 * m + 1) / 2.0L * integ;
                    }
                    B->P[h][k][l] = (double)acc;
                }
        }
    }

    /* sparse weights (App. A): the small faces' subcells are the large face's
       scaled by 1/2, the upper one shifted by +1 */
    for (int h = 0; h < 2; ++h) {
        double tmp[DGO_NMAX * DGO_NMAX];
        dgo_overlap_weights(B->w, n, 0.5, h == 0 ? 0.0 : 1.0, tmp);
        for (int k = 0; k < n; ++k)
            for (int l = 0; l < n; ++l) B->Wt[k][h * n + l] = tmp[k * n + l];
    }
    return 0;
}

/* Overlap lengths of LGL subcells (eq. local_weights, App. A).  The subcell of
   node k of the reference face covers [-1 + sum_{j<k} w_j, -1 + sum_{j<=k} w_j];
   the subcell of node l of the other face covers
   [-1 + shift + scale sum_{j<l} w_j, -1 + shift + scale sum_{j<=l} w_j].
   out[k*n + l] = length of the intersection (0 if they do not overlap). */
void dgo_overlap_weights(const double* wd, int n, double scale, double shift, double* out)
{
    for (int k = 0; k < n; ++k) {
        long double lo_k = -1.0L;
        for (int j = 0; j < k; ++j) lo_k += wd[j];
        long double hi_k = lo_k + wd[k];
        for (int l = 0; l < n; ++l) {
            long double lo_l = -1.0L + shift;
            for (int j = 0; j < l; ++j) lo_l += scale * (long double)wd[j];
            long double hi_l = lo_l + scale * (long double)wd[l];
            long double bl = lo_k > lo_l ? lo_k : lo_l;
            long double bu = hi_k < hi_l ? hi_k : hi_l;
            /* overlaps that vanish in exact arithmetic come out as round-off */
            out[k * n + l] = bu - bl > 1e-12L ? (double)(bu - bl) : 0.0;
        }
    }
}
