/*
 * Oracle for the IDP-limited LGL-DGSEM on 2:1-balanced Cartesian quadtrees.
 *
 * TEST INFRASTRUCTURE ONLY.  This is a plain, slow, FP64 CPU implementation of
 * the method written from the paper ("Invariant-domain-preserving limiting with
 * Adaptive Mesh Refinement for LGL-DGSEM", Bolm, Rueda-Ramirez, Kuzmin,
 * Gassner).  It exists to check the GPU library; only tests, the smoke check
 * and the CPU-baseline leg of the benchmark may load it.  It shares no code,
 * headers or tables with the GPU library.
 *
 * State layout everywhere: u[e][v][b][a], v = (rho, rho v1, rho v2, rho e),
 * a = node index along x, b = node index along y, n = N+1 nodes per direction.
 */
#ifndef DGO_H
#define DGO_H

#include <stdint.h>

#define DGO_NV 4
#define DGO_NMAX 8 /* N <= 7 */

/* ---------------- basis (Sec. 2.1, App. A) ---------------- */
typedef struct {
    int N, n;
    double xi[DGO_NMAX];          /* LGL nodes */
    double w[DGO_NMAX];           /* LGL weights omega_a */
    double D[DGO_NMAX][DGO_NMAX]; /* D[a][k] = phi_k'(xi_a) */
    double S[DGO_NMAX][DGO_NMAX]; /* Sbar = 2 Qbar - Bbar */
    double I[2][DGO_NMAX][DGO_NMAX]; /* I[h][l][k] = phi_k((xi_l -/+ 1)/2) */
    double P[2][DGO_NMAX][DGO_NMAX]; /* P[h][k][l]: L2 projection half h -> full face */
    double Wt[DGO_NMAX][2 * DGO_NMAX]; /* sparse weights, reference measure on [-1,1] */
} dgo_basis;

int dgo_basis_init(dgo_basis* B, int N);
double dgo_lagrange(const dgo_basis* B, int k, double s);
double dgo_legendre(int m, double s);
void dgo_overlap_weights(const double* w, int n, double scale, double shift, double* out);

/* ---------------- Euler (Sec. 3 intro) ---------------- */
void dgo_prim(const double* u, double gamma, double* rho, double* v1, double* v2, double* p);
void dgo_flux_phys(const double* u, int dir, double gamma, double* f);
void dgo_flux_llf(const double* uL, const double* uR, int dir, double gamma, double* f);
void dgo_flux_ranocha(const double* uL, const double* uR, int dir, double gamma, double* f);
void dgo_flux_chandrashekar(const double* uL, const double* uR, int dir, double gamma, double* f);
void dgo_flux_volume(int kind, const double* uL, const double* uR, int dir, double gamma, double* f);
double dgo_lnmean(double x, double y);
double dgo_pressure(const double* u, double gamma);
double dgo_wavespeed(const double* u, int dir, double gamma);

/* ---------------- mesh ---------------- */
enum { FACE_CONF = 0, FACE_SMALL = 1, FACE_LARGE = 2, FACE_BOUNDARY = 3 };
/* boundary conditions of the domain sides (x-, x+, y-, y+) and of boundary nodes:
   reflecting slip wall, characteristic inflow/outflow against an exterior state,
   and plain outflow (the exterior state is the interior one) */
enum { BC_PERIODIC = 0, BC_WALL = 1, BC_CHARACTERISTIC = 2, BC_OUTFLOW = 3 };

typedef struct {
    int type;       /* FACE_CONF / FACE_SMALL / FACE_LARGE */
    int64_t nbr;    /* conforming neighbour element (FACE_CONF) or large element (FACE_SMALL) */
    int64_t mortar; /* mortar id (FACE_SMALL / FACE_LARGE), else -1 */
    int half;       /* FACE_SMALL: 0 = lower half of the large face, 1 = upper */
    int64_t bnode;  /* FACE_BOUNDARY: index of its node 0 among the boundary nodes */
} dgo_face;

typedef struct {
    int64_t large;  /* large element */
    int face;       /* face of the large element: 0=-x 1=+x 2=-y 3=+y */
    int64_t small[2]; /* small elements on the lower / upper half */
} dgo_mortar;

typedef struct {
    dgo_basis B;
    int64_t E;
    int8_t* level;
    int32_t* ix;
    int32_t* iy;
    double x0, y0, Lx, Ly;
    int nx0, ny0;
    double* hx; /* per element */
    double* hy;
    dgo_face* face; /* [E][4] */
    int64_t M;
    dgo_mortar* mort;
    int vflux; /* volume flux: 0 Ranocha, 1 Chandrashekar (Sec. 3.6) */
    int bc[4];      /* per domain side; x- and x+ (y- and y+) periodic together */
    /* boundary nodes, numbered by (element, face, node along the face): the
       condition of each and its exterior state (conservative) */
    int64_t NB;
    int8_t* bkind;
    double* bext; /* [NB][4] */
} dgo_mesh;

int dgo_mesh_build(dgo_mesh* m, int N, int64_t E, const int8_t* level, const int32_t* ix,
                   const int32_t* iy, double x0, double y0, double Lx, double Ly, int nx0,
                   int ny0, char* err, int errlen);
/* the same with boundary conditions bc[4] per side (NULL: all periodic) and
   an exterior state ext[4][4] per side (NULL: zero); every boundary node starts
   with its side's condition and exterior state */
int dgo_mesh_build_bc(dgo_mesh* m, int N, int64_t E, const int8_t* level, const int32_t* ix,
                      const int32_t* iy, double x0, double y0, double Lx, double Ly, int nx0,
                      int ny0, const int* bc, const double* ext, char* err, int errlen);
/* the ghost state of a boundary node with interior state ui on face f */
void dgo_boundary_ghost(int kind, const double* ext, const double* ui, int f, double gamma,
                        double* ug);
void dgo_mesh_release(dgo_mesh* m);

/* ---------------- scheme ---------------- */
typedef struct {
    int64_t fv_inadmissible; /* nodes where the low-order update left the admissible set */
    int64_t violations;      /* nodes outside the bounds after limiting */
    double theta_vol_min, theta_mort_min;
    double alpha_vol_mean, alpha_mort_mean; /* mean of 1-theta over subcell faces / mortars */
    double dt;
} dgo_stats;

enum { RHS_HIGH = 0, RHS_LOW = 1 };
enum { DT_IDP = 0, DT_LOWORDER = 1 };
/* LIM_LOCAL: bounds from bar states (eq. Bounds_Barstates); LIM_LOCAL_LO: from
   the low-order solution (eq. Bounds_LowOrder) */
enum { LIM_NONE = 0, LIM_POSITIVITY = 1, LIM_LOCAL = 2, LIM_COMBINED = 3, LIM_LOCAL_LO = 4 };

int dgo_rhs(const dgo_mesh* m, const double* u, int which, double gamma, double* du);
double dgo_max_dt(const dgo_mesh* m, const double* u, double cfl, int mode, double gamma);
int dgo_fe_step(const dgo_mesh* m, const double* u, double dt, double gamma, double beta,
                int limiter, double* out, dgo_stats* st);
int dgo_ssprk3(const dgo_mesh* m, double* u, double cfl, int mode, double gamma, double beta,
               int limiter, dgo_stats* st);
double dgo_theta_pressure(const double* u0, const double* dc, double pt, double gamma);
/* local limiting (eq. Bounds_Barstates) */
void dgo_bar_state(const double* uL, const double* uR, int dir, double gamma, double* ub);
double dgo_spec_entropy(const double* u, double gamma);
void dgo_local_bounds(const dgo_mesh* m, const double* u, double gamma, double* rlo, double* rhi,
                      double* smin);
double dgo_theta_entropy(const double* u0, const double* dc, double st, double gamma, double thi);
/* local bounds from the low-order solution ufv (eq. Bounds_LowOrder) */
void dgo_lowsol_bounds(const dgo_mesh* m, const double* ufv, double gamma, double* rlo, double* rhi,
                       double* smin);
/* combined limiting (eq. combination_posLim_local): per-element shock
   indicator on the pressure in [0, 1]; a FE step with the indicator given
   (NULL: computed from u) */
void dgo_shock_indicator(const dgo_mesh* m, const double* u, double gamma, double* ind);
int dgo_fe_step_ind(const dgo_mesh* m, const double* u, double dt, double gamma, double beta,
                    int limiter, const double* ind, double* out, dgo_stats* st);
/* the same step, exposing its intermediate results (each may be NULL): uvol
   [E][4][n][n] the state after the volume limiter, before the mortar
   correction; dslot [M][3n][4] per mortar node the difference of the high-order
   and the low-order surface flux terms (Sec. 2.3, in the units of m_i du/dt,
   slots in the order large face, lower small face, upper small face, each by
   face position); theta [M] the mortar factors */
int dgo_fe_step_detail(const dgo_mesh* m, const double* u, double dt, double gamma, double beta,
                       int limiter, const double* ind, double* out, dgo_stats* st, double* uvol,
                       double* dslot, double* theta);
int dgo_ssprk3_dt(const dgo_mesh* m, double* u, double dt, double gamma, double beta, int limiter,
                  dgo_stats* st);

/* ---------------- adaptation (Sec. 2.4), dgo_amr.c ---------------- */
/* new leaf list (capacity 4 E) and its source map: kind 0 kept (src[0] = old
   leaf), 1 child (src[0] = old parent, src[1] = child index cx + 2 cy), 2 parent
   (src[0..3] = old children by child index); returns the new leaf count */
int64_t dgo_adapt(int64_t E, const int8_t* level, const int32_t* ix, const int32_t* iy, int nx0,
                  int ny0, const int8_t* flags, int8_t* nlevel, int32_t* nix, int32_t* niy,
                  int8_t* kind, int64_t* src);
void dgo_transfer(int N, int64_t En, const int8_t* kind, const int64_t* src, const double* uo,
                  double* un);
void dgo_zhang_shu(int N, int64_t En, const int8_t* kind, const int64_t* src, const double* uo,
                   double* un, double eps, double gamma, int64_t* n_limited, int64_t* n_unfixable);

#endif
