/*
 * Oracle: mesh adaptation, solution transfer and the Zhang-Shu transfer
 * limiter (Sec. 2.4).  TEST INFRASTRUCTURE ONLY (see dgo.h).
 *
 * Adaptation rules (integer work; the GPU library's host code implements the
 * same rules independently and must agree bit for bit):
 *  1. A leaf with flag > 0 is refined into its four children.
 *  2. 2:1 face balance: a leaf that would touch a refined leaf's children
 *     across a face while being two levels coarser is refined too, repeated
 *     until nothing changes.  A balanced input needs at most one extra level
 *     per leaf.
 *  3. Four sibling leaves, all with flag < 0 and none refined, are replaced by
 *     their parent if every leaf touching the parent across a face has, after
 *     steps 1-2, a level at most one above the parent's.  Levels before any
 *     coarsening are used, which keeps the result balanced.
 *  4. New leaf order: the old leaves in their order; a kept leaf stays, a
 *     refined leaf becomes its children in the order (0,0), (1,0), (0,1),
 *     (1,1) of (x, y) halves, and a coarsened group becomes its parent at the
 *     position of its first member.
 *
 * Transfer: interpolation of the parent polynomial onto the children's nodes
 * on refinement, exact L2 projection of the four children onto the parent on
 * coarsening (Sec. 2.4).  Both are tensor products of the one-dimensional
 * mortar operators I and P of dgo_basis, so they conserve sum_i m_i u_i.
 *
 * Zhang-Shu limiter (Sec. 2.4, Zhang and Shu 2011): a group (the four children
 * of a refined leaf, or a new parent) is troubled if a node has rho < eps or
 * p < eps.  Then all its nodes are scaled toward the reference mean state ubar,
 * u_i <- ubar + theta (u_i - ubar), with the largest theta in [0, 1] that puts
 * every node at rho >= eps and p >= eps.  The density is aimed at
 * eps (1 + 2^-40), the pressure at eps (1 + 2^-40) + 2^-40 max_i |E_i| over the
 * group's nodes: p = (gamma-1)(E - |m|^2 / (2 rho)) is only known to a few
 * units in the last place of E, and where the kinetic energy dwarfs the
 * pressure (a Mach-2000 jet: E ~ 1e6, p ~ 0.4) a target of eps alone would be
 * crossed by rounding.  The factor from the pressure quadratic can still miss
 * where a node's density becomes small (the quadratic's coefficients cancel at
 * the scale rho_bar E_bar, and p divides that rounding by rho): the scaled
 * states are therefore checked directly, and if one fails, the factor is
 * bisected between 0 (the admissible mean) and the closed-form value.  One theta per group
 * keeps the group's total sum_i m_i u_i.  ubar is the LGL mean of the parent
 * before refinement, or of the projected parent after coarsening.  A group
 * whose mean itself is below the thresholds cannot be fixed: theta = 0.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "dgo.h"

/* ---------------- leaf lookup by (level, ix, iy) ---------------- */
typedef struct {
    uint64_t key;
    int64_t idx;
} kv;

static uint64_t key_of(int l, int64_t ix, int64_t iy)
{
    return ((uint64_t)l << 56) | ((uint64_t)ix << 28) | (uint64_t)iy;
}

static int kv_cmp(const void* a, const void* b)
{
    uint64_t x = ((const kv*)a)->key, y = ((const kv*)b)->key;
    return x < y ? -1 : (x > y ? 1 : 0);
}

static int64_t lookup(const kv* t, int64_t n, int l, int64_t ix, int64_t iy)
{
    uint64_t k = key_of(l, ix, iy);
    int64_t lo = 0, hi = n - 1;
    while (lo <= hi) {
        int64_t mid = (lo + hi) / 2;
        if (t[mid].key == k) return t[mid].idx;
        if (t[mid].key < k) lo = mid + 1;
        else hi = mid - 1;
    }
    return -1;
}

static int64_t wrap(int64_t i, int64_t n) { return ((i % n) + n) % n; }

/* Leaves touching face f (0 -x, 1 +x, 2 -y, 3 +y) of leaf e: the same-level
   neighbour, or the coarser one, or the finer ones.  Returns their count. */
static int face_neighbours(const kv* t, int64_t E, const int8_t* lev, const int32_t* ix,
                           const int32_t* iy, int nx0, int ny0, int64_t e, int f, int64_t out[2])
{
    int l = lev[e];
    int64_t nx = (int64_t)nx0 << l, ny = (int64_t)ny0 << l;
    int64_t jx = ix[e] + (f == 0 ? -1 : (f == 1 ? 1 : 0));
    int64_t jy = iy[e] + (f == 2 ? -1 : (f == 3 ? 1 : 0));
    jx = wrap(jx, nx);
    jy = wrap(jy, ny);
    int64_t s = lookup(t, E, l, jx, jy);
    if (s >= 0) {
        out[0] = s;
        return 1;
    }
    if (l > 0) {
        int64_t c = lookup(t, E, l - 1, jx >> 1, jy >> 1);
        if (c >= 0) {
            out[0] = c;
            return 1;
        }
    }
    /* finer: the two children of cell (jx, jy) adjacent to e */
    int cnt = 0;
    for (int k = 0; k < 2; ++k) {
        int64_t cx, cy;
        if (f < 2) {
            cx = 2 * jx + (f == 0 ? 1 : 0);
            cy = 2 * jy + k;
        } else {
            cx = 2 * jx + k;
            cy = 2 * jy + (f == 2 ? 1 : 0);
        }
        int64_t c = lookup(t, E, l + 1, cx, cy);
        if (c >= 0) out[cnt++] = c;
    }
    return cnt;
}

int64_t dgo_adapt(int64_t E, const int8_t* lev, const int32_t* ix, const int32_t* iy, int nx0,
                  int ny0, const int8_t* flags, int8_t* nlev, int32_t* nix, int32_t* niy,
                  int8_t* kind, int64_t* src)
{
    kv* t = (kv*)malloc(sizeof(kv) * (size_t)(E > 0 ? E : 1));
    for (int64_t e = 0; e < E; ++e) {
        t[e].key = key_of(lev[e], ix[e], iy[e]);
        t[e].idx = e;
    }
    qsort(t, (size_t)E, sizeof(kv), kv_cmp);

    /* steps 1-2: refinement and balance closure */
    char* ref = (char*)calloc((size_t)(E > 0 ? E : 1), 1);
    int changed = 1;
    for (int64_t e = 0; e < E; ++e) ref[e] = flags[e] > 0;
    while (changed) {
        changed = 0;
        for (int64_t e = 0; e < E; ++e) {
            if (ref[e]) continue;
            for (int f = 0; f < 4 && !ref[e]; ++f) {
                int64_t nb[2];
                int c = face_neighbours(t, E, lev, ix, iy, nx0, ny0, e, f, nb);
                for (int k = 0; k < c; ++k)
                    if (lev[nb[k]] + ref[nb[k]] > lev[e] + 1) {
                        ref[e] = 1;
                        changed = 1;
                    }
            }
        }
    }

    /* step 3: coarsening groups; group[e] = first sibling of an accepted group */
    int64_t* group = (int64_t*)malloc(sizeof(int64_t) * (size_t)(E > 0 ? E : 1));
    for (int64_t e = 0; e < E; ++e) group[e] = -1;
    for (int64_t e = 0; e < E; ++e) {
        if (lev[e] == 0 || flags[e] >= 0 || ref[e] || group[e] >= 0) continue;
        int l = lev[e];
        int64_t px = ix[e] >> 1, py = iy[e] >> 1;
        int64_t sib[4];
        int ok = 1;
        for (int c = 0; c < 4 && ok; ++c) {
            sib[c] = lookup(t, E, l, 2 * px + (c & 1), 2 * py + (c >> 1));
            if (sib[c] < 0 || flags[sib[c]] >= 0 || ref[sib[c]]) ok = 0;
        }
        /* every leaf touching the parent across a face: level after
           refinement at most l (= parent level + 1) */
        for (int c = 0; c < 4 && ok; ++c) {
            int cx = c & 1, cy = c >> 1;
            int outer[2] = {cx == 0 ? 0 : 1, cy == 0 ? 2 : 3};
            for (int j = 0; j < 2 && ok; ++j) {
                int64_t nb[2];
                int cnt = face_neighbours(t, E, lev, ix, iy, nx0, ny0, sib[c], outer[j], nb);
                for (int k = 0; k < cnt; ++k)
                    if (lev[nb[k]] + ref[nb[k]] > l) ok = 0;
            }
        }
        if (!ok) continue;
        int64_t first = sib[0];
        for (int c = 1; c < 4; ++c)
            if (sib[c] < first) first = sib[c];
        for (int c = 0; c < 4; ++c) group[sib[c]] = first;
    }

    /* step 4: the new list */
    int64_t n = 0;
    for (int64_t e = 0; e < E; ++e) {
        if (group[e] >= 0) {
            if (group[e] != e) continue;
            int l = lev[e];
            int64_t px = ix[e] >> 1, py = iy[e] >> 1;
            nlev[n] = (int8_t)(l - 1);
            nix[n] = (int32_t)px;
            niy[n] = (int32_t)py;
            kind[n] = 2;
            for (int c = 0; c < 4; ++c) src[n * 4 + c] = lookup(t, E, l, 2 * px + (c & 1), 2 * py + (c >> 1));
            ++n;
        } else if (ref[e]) {
            for (int c = 0; c < 4; ++c) {
                nlev[n] = (int8_t)(lev[e] + 1);
                nix[n] = 2 * ix[e] + (c & 1);
                niy[n] = 2 * iy[e] + (c >> 1);
                kind[n] = 1;
                src[n * 4 + 0] = e;
                src[n * 4 + 1] = c;
                src[n * 4 + 2] = -1;
                src[n * 4 + 3] = -1;
                ++n;
            }
        } else {
            nlev[n] = lev[e];
            nix[n] = ix[e];
            niy[n] = iy[e];
            kind[n] = 0;
            src[n * 4 + 0] = e;
            src[n * 4 + 1] = src[n * 4 + 2] = src[n * 4 + 3] = -1;
            ++n;
        }
    }
    free(t);
    free(ref);
    free(group);
    return n;
}

/* ---------------- transfer ---------------- */
void dgo_transfer(int N, int64_t En, const int8_t* kind, const int64_t* src, const double* uo,
                  double* un)
{
    dgo_basis B;
    dgo_basis_init(&B, N);
    const int n = N + 1, NN = n * n;
    for (int64_t e = 0; e < En; ++e) {
        double* out = un + (size_t)e * 4 * NN;
        if (kind[e] == 0) {
            memcpy(out, uo + (size_t)src[e * 4] * 4 * NN, sizeof(double) * 4 * NN);
        } else if (kind[e] == 1) {
            /* child (cx, cy) of the old parent: value at child node (a, b) is the
               parent polynomial at ((xi_a -/+ 1)/2, (xi_b -/+ 1)/2) */
            const double* p = uo + (size_t)src[e * 4] * 4 * NN;
            int c = (int)src[e * 4 + 1], cx = c & 1, cy = c >> 1;
            for (int v = 0; v < 4; ++v)
                for (int b = 0; b < n; ++b)
                    for (int a = 0; a < n; ++a) {
                        double s = 0.0;
                        for (int l = 0; l < n; ++l)
                            for (int k = 0; k < n; ++k)
                                s += B.I[cy][b][l] * B.I[cx][a][k] * p[(v * n + l) * n + k];
                        out[(v * n + b) * n + a] = s;
                    }
        } else {
            /* parent: L2 projection of the four children, P^{cy} (x) P^{cx} summed */
            for (int i = 0; i < 4 * NN; ++i) out[i] = 0.0;
            for (int c = 0; c < 4; ++c) {
                const double* ch = uo + (size_t)src[e * 4 + c] * 4 * NN;
                int cx = c & 1, cy = c >> 1;
                for (int v = 0; v < 4; ++v)
                    for (int b = 0; b < n; ++b)
                        for (int a = 0; a < n; ++a) {
                            double s = 0.0;
                            for (int l = 0; l < n; ++l)
                                for (int k = 0; k < n; ++k)
                                    s += B.P[cy][b][l] * B.P[cx][a][k] * ch[(v * n + l) * n + k];
                            out[(v * n + b) * n + a] += s;
                        }
            }
        }
    }
}

/* ---------------- Zhang-Shu ---------------- */
#define ZS_MARGIN (1.0 + 0x1p-40)

static void lgl_mean(const dgo_basis* B, const double* u, double* m)
{
    const int n = B->n;
    for (int v = 0; v < 4; ++v) {
        double s = 0.0;
        for (int b = 0; b < n; ++b)
            for (int a = 0; a < n; ++a) s += B->w[a] * B->w[b] * u[(v * n + b) * n + a];
        m[v] = s / 4.0; /* sum of w_a w_b over the element is 4 */
    }
}

/* largest t in [0, 1] with rho >= rt and p >= pt along ubar + t (u - ubar) */
static double zs_theta_node(const double* ub, const double* u, double rt, double pt, double gamma)
{
    double d[4];
    for (int v = 0; v < 4; ++v) d[v] = u[v] - ub[v];
    double t = 1.0;
    if (u[0] < rt) t = (ub[0] - rt) / (ub[0] - u[0]);
    double tp = dgo_theta_pressure(ub, d, pt, gamma);
    return tp < t ? tp : t;
}

/* every node of the group scaled by t toward ubar has rho >= eps and p >= eps */
static int zs_group_ok(const double* un, int64_t first, int64_t cnt, int NN, const double* ub,
                       double t, double eps, double gamma)
{
    for (int64_t g = first; g < first + cnt; ++g)
        for (int q = 0; q < NN; ++q) {
            double w[4];
            for (int v = 0; v < 4; ++v) w[v] = ub[v] + t * (un[((size_t)g * 4 + v) * NN + q] - ub[v]);
            if (!(w[0] >= eps) || !(dgo_pressure(w, gamma) >= eps)) return 0;
        }
    return 1;
}

void dgo_zhang_shu(int N, int64_t En, const int8_t* kind, const int64_t* src, const double* uo,
                   double* un, double eps, double gamma, int64_t* n_limited, int64_t* n_unfixable)
{
    dgo_basis B;
    dgo_basis_init(&B, N);
    const int n = N + 1, NN = n * n;
    const double et = eps * ZS_MARGIN;
    int64_t lim = 0, bad = 0;
    for (int64_t e = 0; e < En; ++e) {
        int64_t first, cnt;
        double ub[4];
        if (kind[e] == 1 && src[e * 4 + 1] == 0) {
            first = e;
            cnt = 4;
            lgl_mean(&B, uo + (size_t)src[e * 4] * 4 * NN, ub);
        } else if (kind[e] == 2) {
            first = e;
            cnt = 1;
            lgl_mean(&B, un + (size_t)e * 4 * NN, ub);
        } else {
            continue;
        }
        int trouble = 0;
        double emax = 0.0;
        for (int64_t g = first; g < first + cnt; ++g)
            for (int q = 0; q < NN; ++q) {
                double w[4];
                for (int v = 0; v < 4; ++v) w[v] = un[((size_t)g * 4 + v) * NN + q];
                double p = dgo_pressure(w, gamma);
                if (!(w[0] >= eps) || !(p >= eps)) trouble = 1;
                if (fabs(w[3]) > emax) emax = fabs(w[3]);
            }
        if (!trouble) continue;
        ++lim;
        const double pt = et + 0x1p-40 * emax;
        double theta;
        if (!(ub[0] > et) || !(dgo_pressure(ub, gamma) > pt)) {
            theta = 0.0;
            ++bad;
        } else {
            theta = 1.0;
            for (int64_t g = first; g < first + cnt; ++g)
                for (int q = 0; q < NN; ++q) {
                    double w[4];
                    for (int v = 0; v < 4; ++v) w[v] = un[((size_t)g * 4 + v) * NN + q];
                    double t = zs_theta_node(ub, w, et, pt, gamma);
                    if (t < theta) theta = t;
                }
            if (!zs_group_ok(un, first, cnt, NN, ub, theta, eps, gamma)) {
                double lo = 0.0, hi = theta;
                for (int it = 0; it < 60; ++it) {
                    const double mid = 0.5 * (lo + hi);
                    if (zs_group_ok(un, first, cnt, NN, ub, mid, eps, gamma)) lo = mid;
                    else hi = mid;
                }
                theta = lo;
            }
        }
        for (int64_t g = first; g < first + cnt; ++g)
            for (int v = 0; v < 4; ++v)
                for (int q = 0; q < NN; ++q) {
                    double* x = &un[((size_t)g * 4 + v) * NN + q];
                    *x = ub[v] + theta * (*x - ub[v]);
                }
    }
    if (n_limited) *n_limited = lim;
    if (n_unfixable) *n_unfixable = bad;
}
