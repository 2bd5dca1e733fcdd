/*
 * Oracle: flat C entry points for the Python test harness (ctypes).
 * TEST INFRASTRUCTURE ONLY (see dgo.h).
 */
#include <stdlib.h>
#include <string.h>

#include "dgo.h"

#ifdef _OPENMP
#include <omp.h>
#endif

int orc_basis(int N, double* xi, double* w, double* D, double* S)
{
    dgo_basis B;
    if (dgo_basis_init(&B, N)) return -1;
    int n = N + 1;
    for (int i = 0; i < n; ++i) {
        xi[i] = B.xi[i];
        w[i] = B.w[i];
        for (int j = 0; j < n; ++j) {
            D[i * n + j] = B.D[i][j];
            S[i * n + j] = B.S[i][j];
        }
    }
    return 0;
}

/* I: [2][n][n] (h, l, k), P: [2][n][n] (h, k, l), Wt: [n][2n] */
int orc_mortar_ops(int N, double* I, double* P, double* Wt)
{
    dgo_basis B;
    if (dgo_basis_init(&B, N)) return -1;
    int n = N + 1;
    for (int h = 0; h < 2; ++h)
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                I[(h * n + i) * n + j] = B.I[h][i][j];
                P[(h * n + i) * n + j] = B.P[h][i][j];
            }
    for (int k = 0; k < n; ++k)
        for (int j = 0; j < 2 * n; ++j) Wt[k * 2 * n + j] = B.Wt[k][j];
    return 0;
}

double orc_lagrange(int N, int k, double s)
{
    dgo_basis B;
    dgo_basis_init(&B, N);
    return dgo_lagrange(&B, k, s);
}

double orc_legendre(int m, double s) { return dgo_legendre(m, s); }

void orc_flux(int kind, const double* uL, const double* uR, int dir, double gamma, double* f)
{
    if (kind == 0) dgo_flux_phys(uL, dir, gamma, f);
    else if (kind == 1) dgo_flux_llf(uL, uR, dir, gamma, f);
    else if (kind == 2) dgo_flux_ranocha(uL, uR, dir, gamma, f);
    else dgo_flux_chandrashekar(uL, uR, dir, gamma, f);
}

double orc_lnmean(double x, double y) { return dgo_lnmean(x, y); }

void* orc_mesh_new(int N, int64_t E, const int8_t* level, const int32_t* ix, const int32_t* iy,
                   double x0, double y0, double Lx, double Ly, int nx0, int ny0, char* err,
                   int errlen)
{
    dgo_mesh* m = (dgo_mesh*)malloc(sizeof(dgo_mesh));
    if (dgo_mesh_build(m, N, E, level, ix, iy, x0, y0, Lx, Ly, nx0, ny0, err, errlen)) {
        dgo_mesh_release(m);
        free(m);
        return 0;
    }
    return m;
}

void orc_mesh_free(void* h)
{
    dgo_mesh* m = (dgo_mesh*)h;
    if (!m) return;
    dgo_mesh_release(m);
    free(m);
}

void* orc_mesh_new_bc(int N, int64_t E, const int8_t* level, const int32_t* ix, const int32_t* iy,
                      double x0, double y0, double Lx, double Ly, int nx0, int ny0, const int* bc,
                      const double* ext, char* err, int errlen)
{
    dgo_mesh* m = (dgo_mesh*)malloc(sizeof(dgo_mesh));
    if (dgo_mesh_build_bc(m, N, E, level, ix, iy, x0, y0, Lx, Ly, nx0, ny0, bc, ext, err, errlen)) {
        dgo_mesh_release(m);
        free(m);
        return 0;
    }
    return m;
}

int64_t orc_mesh_num_mortars(void* h) { return ((dgo_mesh*)h)->M; }

int64_t orc_mesh_num_bnodes(void* h) { return ((dgo_mesh*)h)->NB; }

/* boundary nodes: [NB][3] of (element, face, node along the face) */
void orc_mesh_boundary_nodes(void* h, int64_t* out)
{
    dgo_mesh* m = (dgo_mesh*)h;
    for (int64_t e = 0; e < m->E; ++e)
        for (int f = 0; f < 4; ++f) {
            const dgo_face* F = &m->face[e * 4 + f];
            if (F->type != FACE_BOUNDARY) continue;
            for (int k = 0; k < m->B.n; ++k) {
                out[(F->bnode + k) * 3 + 0] = e;
                out[(F->bnode + k) * 3 + 1] = f;
                out[(F->bnode + k) * 3 + 2] = k;
            }
        }
}

/* per boundary node condition (BC_WALL, BC_CHARACTERISTIC, BC_OUTFLOW) and
   exterior state; -1 if a condition is out of range */
int orc_mesh_set_boundary_states(void* h, const int8_t* kind, const double* ext)
{
    dgo_mesh* m = (dgo_mesh*)h;
    for (int64_t j = 0; j < m->NB; ++j)
        if (kind[j] < BC_WALL || kind[j] > BC_OUTFLOW) return -1;
    for (int64_t j = 0; j < m->NB; ++j) {
        m->bkind[j] = kind[j];
        for (int v = 0; v < 4; ++v) m->bext[j * 4 + v] = ext[j * 4 + v];
    }
    return 0;
}

void orc_boundary_ghost(int kind, const double* ext, const double* ui, int f, double gamma,
                        double* ug)
{
    dgo_boundary_ghost(kind, ext, ui, f, gamma, ug);
}

void orc_mesh_set_volume_flux(void* h, int kind) { ((dgo_mesh*)h)->vflux = kind; }

/* face table: [E][4] of (type, nbr, mortar, half) */
void orc_mesh_faces(void* h, int64_t* out)
{
    dgo_mesh* m = (dgo_mesh*)h;
    for (int64_t i = 0; i < m->E * 4; ++i) {
        out[i * 4 + 0] = m->face[i].type;
        out[i * 4 + 1] = m->face[i].nbr;
        out[i * 4 + 2] = m->face[i].mortar;
        out[i * 4 + 3] = m->face[i].half;
    }
}

/* mortars: [M] of (large, face, small0, small1) */
void orc_mesh_mortars(void* h, int64_t* out)
{
    dgo_mesh* m = (dgo_mesh*)h;
    for (int64_t s = 0; s < m->M; ++s) {
        out[s * 4 + 0] = m->mort[s].large;
        out[s * 4 + 1] = m->mort[s].face;
        out[s * 4 + 2] = m->mort[s].small[0];
        out[s * 4 + 3] = m->mort[s].small[1];
    }
}

/* node coordinates and masses, [E][n][n] each (b, a) */
void orc_mesh_geometry(void* h, double* x, double* y, double* mass)
{
    dgo_mesh* m = (dgo_mesh*)h;
    int n = m->B.n;
    for (int64_t e = 0; e < m->E; ++e) {
        double xl = m->x0 + m->ix[e] * m->hx[e], yl = m->y0 + m->iy[e] * m->hy[e];
        for (int b = 0; b < n; ++b)
            for (int a = 0; a < n; ++a) {
                int64_t i = (e * n + b) * n + a;
                x[i] = xl + (m->B.xi[a] + 1.0) * 0.5 * m->hx[e];
                y[i] = yl + (m->B.xi[b] + 1.0) * 0.5 * m->hy[e];
                mass[i] = m->hx[e] * m->hy[e] / 4.0 * m->B.w[a] * m->B.w[b];
            }
    }
}

int orc_rhs(void* h, const double* u, int which, double gamma, double* du)
{
    return dgo_rhs((dgo_mesh*)h, u, which, gamma, du);
}

double orc_max_dt(void* h, const double* u, double cfl, int mode, double gamma)
{
    return dgo_max_dt((dgo_mesh*)h, u, cfl, mode, gamma);
}

/* stats out: [fv_inadmissible, violations, theta_vol_min, theta_mort_min,
               alpha_vol_mean, alpha_mort_mean, dt] */
static void pack(const dgo_stats* s, double* o)
{
    o[0] = (double)s->fv_inadmissible;
    o[1] = (double)s->violations;
    o[2] = s->theta_vol_min;
    o[3] = s->theta_mort_min;
    o[4] = s->alpha_vol_mean;
    o[5] = s->alpha_mort_mean;
    o[6] = s->dt;
}

int orc_fe_step(void* h, const double* u, double dt, double gamma, double beta, int limiter,
                double* out, double* stats)
{
    dgo_stats s;
    int rc = dgo_fe_step((dgo_mesh*)h, u, dt, gamma, beta, limiter, out, &s);
    pack(&s, stats);
    return rc;
}

int orc_ssprk3(void* h, double* u, double cfl, int mode, double gamma, double beta, int limiter,
               double* stats)
{
    dgo_stats s;
    int rc = dgo_ssprk3((dgo_mesh*)h, u, cfl, mode, gamma, beta, limiter, &s);
    pack(&s, stats);
    return rc;
}

int orc_ssprk3_dt(void* h, double* u, double dt, double gamma, double beta, int limiter,
                  double* stats)
{
    dgo_stats s;
    int rc = dgo_ssprk3_dt((dgo_mesh*)h, u, dt, gamma, beta, limiter, &s);
    pack(&s, stats);
    return rc;
}

void orc_overlap_weights(int N, double scale, double shift, double* out)
{
    dgo_basis B;
    dgo_basis_init(&B, N);
    dgo_overlap_weights(B.w, N + 1, scale, shift, out);
}

double orc_theta_pressure(const double* u0, const double* dc, double pt, double gamma)
{
    return dgo_theta_pressure(u0, dc, pt, gamma);
}

void orc_bar_state(const double* uL, const double* uR, int dir, double gamma, double* ub)
{
    dgo_bar_state(uL, uR, dir, gamma, ub);
}

double orc_spec_entropy(const double* u, double gamma) { return dgo_spec_entropy(u, gamma); }

double orc_theta_entropy(const double* u0, const double* dc, double st, double gamma, double thi)
{
    return dgo_theta_entropy(u0, dc, st, gamma, thi);
}

void orc_local_bounds(void* h, const double* u, double gamma, double* rlo, double* rhi, double* smin)
{
    dgo_local_bounds((dgo_mesh*)h, u, gamma, rlo, rhi, smin);
}

void orc_lowsol_bounds(void* h, const double* ufv, double gamma, double* rlo, double* rhi,
                       double* smin)
{
    dgo_lowsol_bounds((dgo_mesh*)h, ufv, gamma, rlo, rhi, smin);
}

void orc_shock_indicator(void* h, const double* u, double gamma, double* ind)
{
    dgo_shock_indicator((dgo_mesh*)h, u, gamma, ind);
}

int orc_fe_step_ind(void* h, const double* u, double dt, double gamma, double beta, int limiter,
                    const double* ind, double* out, double* stats)
{
    dgo_stats s;
    int rc = dgo_fe_step_ind((dgo_mesh*)h, u, dt, gamma, beta, limiter, ind, out, &s);
    pack(&s, stats);
    return rc;
}

int orc_fe_step_detail(void* h, const double* u, double dt, double gamma, double beta, int limiter,
                       double* out, double* stats, double* uvol, double* dslot, double* theta)
{
    dgo_stats s;
    int rc = dgo_fe_step_detail((dgo_mesh*)h, u, dt, gamma, beta, limiter, 0, out, &s, uvol, dslot, theta);
    pack(&s, stats);
    return rc;
}

int orc_set_threads(int t)
{
#ifdef _OPENMP
    if (t > 0) omp_set_num_threads(t);
    return omp_get_max_threads();
#else
    (void)t;
    return 1;
#endif
}

int64_t orc_adapt(int64_t E, const int8_t* level, const int32_t* ix, const int32_t* iy, int nx0,
                  int ny0, const int8_t* flags, int8_t* nlevel, int32_t* nix, int32_t* niy,
                  int8_t* kind, int64_t* src)
{
    return dgo_adapt(E, level, ix, iy, nx0, ny0, flags, nlevel, nix, niy, kind, src);
}

void orc_transfer(int N, int64_t En, const int8_t* kind, const int64_t* src, const double* uo,
                  double* un, double eps, double gamma, int64_t* counts)
{
    dgo_transfer(N, En, kind, src, uo, un);
    if (eps > 0.0) dgo_zhang_shu(N, En, kind, src, uo, un, eps, gamma, &counts[0], &counts[1]);
    else counts[0] = counts[1] = 0;
}
