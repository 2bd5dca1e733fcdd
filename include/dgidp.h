/*
 * dgidp: MI355X (gfx950) library for the invariant-domain-preserving (IDP)
 * limited LGL-DGSEM of the 2D compressible Euler equations on 2:1-balanced
 * Cartesian quadtrees, periodic or with slip-wall, characteristic or outflow
 * sides (Bolm, Rueda-Ramirez, Kuzmin, Gassner:
 * "Invariant-domain-preserving limiting with Adaptive Mesh Refinement for
 * Legendre-Gauss-Lobatto Discontinuous Galerkin Spectral Element Methods").
 *
 * Conventions shared by every entry point
 *  - Return value: 0 on success, a negative DGIDP_E_* code on failure.  No
 *    entry point aborts the process.  After an error the context stays usable,
 *    except after DGIDP_E_DEVICE.  dgidp_last_error() gives a message.
 *  - Nodal state layout (external order): u[e][v][j][i], e = leaf index in the
 *    caller's leaf order, v = (rho, rho v1, rho v2, rho e), j = LGL node index
 *    along y, i = LGL node index along x, N+1 nodes per direction.
 *  - Pointers flagged `on_device` are device pointers used on the context's
 *    stream; otherwise they are host pointers.  The caller owns every pointer
 *    it passes; the library copies what it keeps.  The context owns all device
 *    buffers it allocates.
 *  - Asynchrony: entry points that take no host output pointer only enqueue
 *    work on the context's stream; those that return host values synchronise.
 *  - Host threads: a context is not thread-safe; the caller serialises the
 *    calls on one context.  Distinct contexts own distinct buffers and may be
 *    driven from different threads; they share only the read-only basis
 *    tables in device constant memory, which dgidp_create writes with the
 *    same values for a given N.
 */
#ifndef DGIDP_H
#define DGIDP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    DGIDP_OK = 0,
    DGIDP_E_INVALID_ARG = -1,
    DGIDP_E_UNSUPPORTED_N = -2,
    DGIDP_E_DEVICE = -3,
    DGIDP_E_MESH_GAP_OR_OVERLAP = -4,
    DGIDP_E_MESH_NOT_BALANCED = -5,
    DGIDP_E_STATE_INADMISSIBLE = -6,
    DGIDP_E_NO_MESH = -7,
    DGIDP_E_NO_STATE = -8,
    DGIDP_E_DT = -9
};

enum { DGIDP_FP64 = 0, DGIDP_MIXED = 1 };           /* precision of the high-order fluxes */
enum { DGIDP_DT_IDP = 0, DGIDP_DT_LOWORDER = 1 };   /* time-step rule */
enum {
    DGIDP_LIMIT_NONE = 0,
    DGIDP_LIMIT_POSITIVITY = 1,
    DGIDP_LIMIT_LOCAL = 2,
    DGIDP_LIMIT_COMBINED = 3,
    DGIDP_LIMIT_LOCAL_LOWORDER = 4
};
enum { DGIDP_RHS_HIGH = 0, DGIDP_RHS_LOW = 1 };
enum { DGIDP_FLUX_RANOCHA = 0, DGIDP_FLUX_CHANDRASHEKAR = 1 };  /* two-point volume flux */
/* boundary condition of a domain side or boundary node */
enum { DGIDP_BC_PERIODIC = 0, DGIDP_BC_WALL = 1, DGIDP_BC_CHARACTERISTIC = 2, DGIDP_BC_OUTFLOW = 3 };

typedef struct dgidp_ctx dgidp_ctx;

/* Parameters of the scheme.
 *  N          polynomial degree (GPU kernels exist for N = 3 and N = 4)
 *  gamma      ratio of specific heats (Sec. 3: 1.4; 3 in Sec. 3.2)
 *  beta       positivity bound factor: rho >= beta rho^FV, p >= beta p^FV
 *             (eq. Bounds_Positivity, beta = 0.1)
 *  precision  DGIDP_FP64, or DGIDP_MIXED: FP32 volume flux differencing and
 *             mortar interpolation/projection, FP64 everything else
 *  dt_mode    DGIDP_DT_IDP (eq. timestep_restriction) or DGIDP_DT_LOWORDER
 *             (eq. CFLcondition_lowordermethod, constant of the standard
 *             DGSEM estimate: dt = CFL / max_i (N+1)(lambda_1/hx + lambda_2/hy))
 *  limiter    DGIDP_LIMIT_NONE (pure high order), DGIDP_LIMIT_POSITIVITY
 *             (Sec. 2.3: volume then mortar convex limiting against
 *             eq. Bounds_Positivity) or DGIDP_LIMIT_LOCAL (the same, plus the
 *             local bounds of eq. Bounds_Barstates: per node the minimum and
 *             maximum density and the minimum specific entropy p rho^-gamma
 *             over the node and the bar states of its low-order neighbours,
 *             taken from the stage's input state; the density floor is the
 *             larger of the local and the positivity floor), or
 *             DGIDP_LIMIT_COMBINED (Sec. 3.5, eq. combination_posLim_local:
 *             per subcell face alpha = (1 - w) alpha_pos + w alpha_local with w
 *             the element's Hennemann indicator on the pressure in [0, 1],
 *             computed from each stage's input; per mortar w is the largest
 *             indicator of its three elements; only the positivity bounds
 *             are guaranteed), or DGIDP_LIMIT_LOCAL_LOWORDER (Sec. 3.4,
 *             eq. Bounds_LowOrder: as DGIDP_LIMIT_LOCAL, with the bounds
 *             taken over the low-order solution u + dt R_LO / m of the node
 *             and its low-order neighbours instead of the bar states; no
 *             neighbour across a boundary; the entropy bound only from
 *             low-order states with positive density and pressure; meant
 *             for the low-order CFL rule, under which it is not provably
 *             bound-preserving)
 *  strict_dt  if nonzero, dgidp_limit() rejects a dt above the IDP bound
 *  volume_flux  two-point flux of the volume flux differencing:
 *             DGIDP_FLUX_RANOCHA (Ranocha's entropy-conserving, kinetic-energy-
 *             preserving flux, Sec. 3 intro; 0, the default of a zeroed struct)
 *             or DGIDP_FLUX_CHANDRASHEKAR (Chandrashekar's, Sec. 3.6) */
typedef struct {
    int N;
    double gamma;
    double beta;
    int precision;
    int dt_mode;
    int limiter;
    int strict_dt;
    int volume_flux;
} dgidp_params;

/* Statistics of one limited forward-Euler step or one SSP-RK3 step (summed or
 * reduced over its stages).  alpha = 1 - theta is the low-order fraction
 * (Sec. 3 intro: alpha = 1 pure low order). */
typedef struct {
    int64_t fv_inadmissible; /* nodes whose low-order update left rho > 0, p > 0 */
    int64_t violations;      /* nodes outside the bounds after limiting: the positivity
                                bounds with tolerance 0; the local bounds within a
                                relative 1e-12 (the low-order state meets them only
                                up to rounding) */
    double theta_vol_min;    /* smallest volume blending factor */
    double theta_mort_min;   /* smallest mortar blending factor */
    double alpha_vol_mean;   /* mean of 1 - theta over interior subcell faces */
    double alpha_mort_mean;  /* mean of 1 - theta over mortars */
    double dt;               /* time step used */
} dgidp_stats;

/* Create a context.  `stream` is a hipStream_t (may be NULL for the null
 * stream), borrowed, e.g. torch.cuda.current_stream().cuda_stream.
 * Errors: DGIDP_E_INVALID_ARG, DGIDP_E_UNSUPPORTED_N, DGIDP_E_DEVICE. */
int dgidp_create(const dgidp_params* p, void* stream, dgidp_ctx** out);
void dgidp_destroy(dgidp_ctx* ctx);
const char* dgidp_last_error(dgidp_ctx* ctx);
int dgidp_set_stream(dgidp_ctx* ctx, void* stream);
int dgidp_synchronize(dgidp_ctx* ctx);

/* Upload a quadtree mesh (Sec. 3.1: leaves are the elements).  The root grid
 * is nx0 x ny0 on [x0, x0+Lx] x [y0, y0+Ly], periodic in both directions
 * unless dgidp_set_boundaries said otherwise; leaf
 * e covers cell (ix[e], iy[e]) of the (nx0 2^level[e]) x (ny0 2^level[e]) grid.
 * Neighbours across a face may differ by one level (Sec. 2.2: 2-to-1
 * nonconforming interfaces).  Host arrays, copied.  Replaces any previous mesh
 * and state.  The device buffers of a mesh are kept by the context and reused
 * by later meshes and adaptations (grown when a mesh needs more); only
 * dgidp_destroy releases them.  Limits: level[e] in 0..20, and 1 <= n_leaves <=
 * 2^30 / (4 (N+1)^2) (16,777,216 at N = 3, 10,737,418 at N = 4), since the
 * kernels index state values with 32-bit integers.  Errors:
 * DGIDP_E_MESH_GAP_OR_OVERLAP (leaves do not tile the domain, or a leaf lies
 * outside the root grid or above level 20), DGIDP_E_MESH_NOT_BALANCED,
 * DGIDP_E_INVALID_ARG (n_leaves outside its limits, NULL arrays, an empty root
 * grid). */
int dgidp_mesh_upload(dgidp_ctx* ctx, int64_t n_leaves, const int8_t* level, const int32_t* ix,
                      const int32_t* iy, double x0, double y0, double Lx, double Ly, int nx0,
                      int ny0);
/* Host-only: validate a leaf list like dgidp_mesh_upload on a periodic domain
 * (same errors, message in msg) without a context or GPU; returns the number
 * of mortars and of nodes that lie on two mortars.  Output pointers may be
 * NULL. */
int dgidp_mesh_validate(int N, int64_t n_leaves, const int8_t* level, const int32_t* ix,
                        const int32_t* iy, int nx0, int ny0, int64_t* n_mortars,
                        int64_t* n_two_mortar_nodes, char* msg, int msglen);
/* The same with the side conditions bc[4] of dgidp_set_boundaries (NULL: all
 * periodic): faces on non-periodic sides need no partner across the domain
 * boundary.  Also returns the number of boundary nodes (n_boundary_nodes, may
 * be NULL).  Errors as dgidp_mesh_validate, and DGIDP_E_INVALID_ARG for an
 * unknown condition or opposite sides that disagree on periodicity. */
int dgidp_mesh_validate_bc(int N, int64_t n_leaves, const int8_t* level, const int32_t* ix,
                           const int32_t* iy, int nx0, int ny0, const int* bc, int64_t* n_mortars,
                           int64_t* n_boundary_nodes, char* msg, int msglen);
/* Boundary conditions of the domain sides, in the order x-, x+, y-, y+ (the
 * double Mach reflection (Sec. 3.5) and the jet (Sec. 3.6) use slip walls and
 * characteristic inflow/outflow).  bc[4]: DGIDP_BC_PERIODIC, DGIDP_BC_WALL
 * (reflecting slip wall), DGIDP_BC_CHARACTERISTIC (inflow/outflow against an
 * exterior state) or DGIDP_BC_OUTFLOW (the exterior state is the interior
 * one); opposite sides are periodic together or not at all.  ext: host array
 * [4][4], the conservative exterior state of each side (read for
 * characteristic sides, which need it admissible; may be NULL if there are
 * none).  A boundary node's surface flux, low-order flux, bar state and local
 * bounds use the LLF flux against its ghost state: a wall mirrors the normal
 * momentum; a characteristic node, by the outward normal velocity vn and the
 * sound speed c of its interior state, takes the exterior state (vn <= -c),
 * the exterior density and velocity with the interior pressure (-c < vn <= 0),
 * the interior density and velocity with the exterior pressure (0 < vn < c),
 * or the interior state (vn >= c).  Call before dgidp_mesh_upload; the
 * setting holds for later uploads and adaptations of this context (default:
 * periodic).  Mesh adaptation balances leaves as on a periodic domain, which
 * can refine a few leaves more than needed next to a boundary.  Errors:
 * DGIDP_E_INVALID_ARG (unknown condition, mixed periodicity, inadmissible
 * exterior state, a mesh already uploaded). */
int dgidp_set_boundaries(dgidp_ctx* ctx, const int* bc, const double* ext);
/* Boundary nodes of the uploaded mesh: *n_nodes, and if nodes is not NULL the
 * host array [n_nodes][3] of (element, face, node along the face), numbered by
 * element (external order), then face, then node (in the direction of the
 * face's coordinate).  Errors: DGIDP_E_NO_MESH. */
int dgidp_boundary_nodes(dgidp_ctx* ctx, int64_t* n_nodes, int64_t* nodes);
/* Per boundary node condition (DGIDP_BC_WALL, _CHARACTERISTIC or _OUTFLOW) and
 * conservative exterior state, host arrays [n_nodes] and [n_nodes][4] in the
 * numbering of dgidp_boundary_nodes; copied to the device after the stream's
 * pending work.  A mesh upload or adaptation resets them to the side settings.
 * Errors: DGIDP_E_NO_MESH, DGIDP_E_INVALID_ARG (unknown condition,
 * inadmissible exterior state of a characteristic node; nothing is changed). */
int dgidp_set_boundary_states(dgidp_ctx* ctx, const int8_t* kind, const double* ext);
/* Number of elements and of mortars (nonconforming faces) of the mesh. */
int dgidp_mesh_info(dgidp_ctx* ctx, int64_t* n_elements, int64_t* n_mortars);
/* Physical node coordinates, host arrays [E][N+1][N+1] (external order). */
int dgidp_node_coords(dgidp_ctx* ctx, double* x, double* y);

/* Upload / download the nodal state (layout above).  Upload checks that every
 * value is finite and rho > 0, p > 0 (DGIDP_E_STATE_INADMISSIBLE, first bad
 * node in the message). */
int dgidp_state_upload(dgidp_ctx* ctx, const double* u, int on_device);
int dgidp_state_download(dgidp_ctx* ctx, double* u, int on_device);
/* Failure detection: check the context's current state on the device against
 * the admissible set (every value finite, rho > 0, p > 0; the set that the
 * limiter keeps, Sec. 2.2 and eq. Bounds_Positivity).  *first_bad = -1 if every
 * node is admissible, else element * (N+1)^2 + node (external element order) of
 * one inadmissible node: the first one in the library's internal order.
 * Synchronises.  Errors: DGIDP_E_NO_STATE. */
int dgidp_state_check(dgidp_ctx* ctx, int64_t* first_bad);

/* Semi-discrete time derivative du/dt of the current state (eq. evolutionformula
 * with Kopriva's L2 mortars for DGIDP_RHS_HIGH; eq. FVmethod with the sparse IDP
 * mortar flux of eq. interfaceflux_local for DGIDP_RHS_LOW); no limiting.
 * Same layout as the state. */
int dgidp_rhs(dgidp_ctx* ctx, int which, double* du, int on_device);

/* Largest stable time step times cfl (dt_mode of the context; eq.
 * timestep_restriction for DGIDP_DT_IDP).  Synchronises. */
int dgidp_max_dt(dgidp_ctx* ctx, double cfl, double* dt);

/* One limited forward-Euler step of size dt, in place (Sec. 2.3: low-order
 * update, volume correction, mortar correction).  `s` may be NULL (then the
 * call only enqueues work).  Errors: DGIDP_E_DT in strict mode. */
int dgidp_limit(dgidp_ctx* ctx, double dt, dgidp_stats* s);

/* One SSP-RK3 step in place (Shu-Osher form, each stage a limited forward-Euler
 * step), dt = cfl times the bound of the context's dt_mode, evaluated once at
 * the start of the step.  dt_used and s may be NULL (then nothing is copied to
 * the host and the call only enqueues work). */
int dgidp_step(dgidp_ctx* ctx, double cfl, double* dt_used, dgidp_stats* s);
/* enable != 0: enqueue-only steps (dt_used and s both NULL) replay a HIP graph
 * of the step's kernels, captured on first use per cfl (and per internal
 * time-step accumulator); results are identical to kernel-by-kernel launches.
 * Default: disabled (on the 22k-element blast a replayed step took 107 us
 * against 102 us for direct launches). */
int dgidp_set_graphs(dgidp_ctx* ctx, int enable);
/* Same with a given dt (used to land exactly on an end time). */
int dgidp_step_dt(dgidp_ctx* ctx, double dt, dgidp_stats* s);
/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): one SSP-RK3
 * step in place, the same as dgidp_step(ctx, cfl, NULL, NULL), that allocates
 * nothing.  Its per-step buffers (the two stage states, the mortar slot records,
 * the dt accumulators and dt, the combined-limiting indicator and the
 * low-order-bounds arrays) live in one static device array per GPU of 64 MiB
 * (kept until the process ends), set up when a context is created.  Limit: the
 * buffers of the mesh must fit, about 2 x 32 B per node plus 128 B per mortar
 * node (plus 72 B per node with DGIDP_LIMIT_LOCAL_LOWORDER): up to about 1.0
 * million nodes, for example 65,000 elements at N = 3 or 41,000 at N = 4;
 * larger meshes return DGIDP_E_INVALID_ARG with the required size in the
 * message, and nothing is enqueued.  Enqueue only (no statistics, no host
 * synchronisation); the result equals dgidp_step's bit for bit.  Every call
 * on a GPU shares that GPU's array: calls that overlap on one GPU (on several
 * streams or host threads) race and must be serialised by the caller.  The
 * device current on the calling thread must be the context's device. */
int dgidp_step_noalloc(dgidp_ctx* ctx, double cfl);

/* ---------------- adaptive mesh refinement (Sec. 2.4) ---------------- */

/* Counts of one adaptation. */
typedef struct {
    int64_t n_refined;         /* old leaves replaced by four children (flagged or balance) */
    int64_t n_balance_refined; /* of those, refined only to keep 2:1 balance */
    int64_t n_coarsened;       /* sibling groups replaced by their parent */
    int64_t zs_limited;        /* transferred groups the Zhang-Shu limiter scaled */
    int64_t zs_unfixable;      /* of those, groups whose mean is below the threshold */
} dgidp_adapt_stats;

/* Host-only: the leaf list after refine / coarsen flags (+1 refine, -1 ask to
 * coarsen, 0 keep; one per leaf, external order), without a context.
 * Rules: flagged leaves are refined; a leaf that would end up two levels
 * coarser than a face neighbour is refined too (repeated until stable); four
 * sibling leaves all flagged -1 and none refined are merged into their parent
 * if every leaf touching the parent across a face is at most one level finer
 * than the parent.  New order: the old order with a refined leaf replaced by
 * its children (x half fastest: (0,0) (1,0) (0,1) (1,1)) and a merged group by
 * its parent at the place of its first member.  Source map per new leaf:
 * kind 0 kept (src[0] old leaf), 1 child (src[0] old parent, src[1] child
 * index), 2 parent (src[0..3] old children by child index); src is [n][4].
 * With new_level == NULL only *n_new is returned.  Errors:
 * DGIDP_E_INVALID_ARG (also when capacity < *n_new). */
int dgidp_adapt_leaves(int64_t n_leaves, const int8_t* level, const int32_t* ix, const int32_t* iy,
                       int nx0, int ny0, const int8_t* flags, int64_t capacity, int8_t* new_level,
                       int32_t* new_ix, int32_t* new_iy, int8_t* kind, int64_t* src,
                       int64_t* n_new);

/* Adapt the context's mesh by the host array `flags` (rules of
 * dgidp_adapt_leaves) and transfer the state (Sec. 2.4): interpolation onto
 * children, exact L2 projection onto merged parents, then, if zs_eps > 0, the
 * Zhang-Shu scaling limiter on every transferred group (four children, or one
 * parent) that has a node with rho < zs_eps or p < zs_eps: all its nodes are
 * scaled toward the parent's mean (before refinement) or the projected mean
 * (after coarsening) by the largest common factor that restores the
 * thresholds, which keeps the group's mass.  The new leaf order is that of
 * dgidp_adapt_leaves; dgidp_mesh_download returns it.  Synchronises.
 * Errors: DGIDP_E_NO_STATE, DGIDP_E_INVALID_ARG, DGIDP_E_DEVICE (after which
 * the context may hold the new mesh without a state). */
int dgidp_refine_coarsen(dgidp_ctx* ctx, const int8_t* flags, double zs_eps, int64_t* n_leaves_out,
                         dgidp_adapt_stats* st);
/* The current leaf list (external order), host arrays of mesh_info's size. */
int dgidp_mesh_download(dgidp_ctx* ctx, int8_t* level, int32_t* ix, int32_t* iy);

/* Host-only three-level controller: target level = max_level where
 * indicator >= max_threshold, else med_level where indicator >= med_threshold,
 * else base_level; flag = +1 below the target, -1 above it, 0 at it. */
int dgidp_amr_flags(int64_t n, const float* indicator, const int8_t* level, int base_level,
                    int med_level, float med_threshold, int max_level, float max_threshold,
                    int8_t* flags);

/* ---------------- troubled-cell / AMR indicators ---------------- */

enum { DGIDP_IND_HENNEMANN = 0, DGIDP_IND_MLP = 1 };
#define DGIDP_MLP_NPARAM 5313

/* Per-element indicator of the current state, FP32 [E], external order.
 * DGIDP_IND_HENNEMANN: the modal shock indicator of Hennemann et al. (the
 * paper's AMR indicator for shocks, Sec. 3.3 to 3.6) on rho p: orthonormal
 * Legendre modes, energy = max of the energy fractions of the highest and the
 * second-highest mode shells, alpha = 1 / (1 + exp(-(s/T)(energy - T))) with
 * T = 0.5 10^(-1.8 (N+1)^(1/4)), s = ln(9999); alpha < 1e-3 -> 0; capped at 0.5.
 * DGIDP_IND_MLP: the learned network of dgidp_mlp_* applied to the features of
 * dgidp_features (its raw output).  Errors: DGIDP_E_NO_STATE,
 * DGIDP_E_INVALID_ARG (unknown kind, network weights not set). */
int dgidp_indicator(dgidp_ctx* ctx, int kind, float* alpha, int on_device);
/* The 16 learned-indicator features per element, FP32 [E][16], external
 * order: for q = rho, then p, the x-shell energy fractions sum_j m_kj^2 / E_q
 * and then the y-shell fractions sum_i m_ik^2 / E_q of the orthonormal
 * Legendre modes m of q, shells k = N-3 .. N. */
int dgidp_features(dgidp_ctx* ctx, float* f, int on_device);

/* Learned indicator network, 16 -> 64 -> 64 -> 1, ReLU, for the callers that
 * want a cheaper or trained AMR indicator.  Parameters, FP32, in this order:
 * W1[64][16], b1[64], W2[64][64], b2[64], W3[64], b3 (W[j][k]: unit j, input
 * k), DGIDP_MLP_NPARAM values.  The context keeps FP32 master weights and a
 * BF16 copy (round to nearest even) that every pass uses.  Inference
 * (dgidp_mlp_forward, DGIDP_IND_MLP) multiplies BF16 operands with FP32
 * accumulation: the inputs and the first hidden layer are rounded to BF16
 * (nearest even) before their products; biases, ReLU and the output layer are
 * FP32.  Training (grad, train_step) runs in FP32 arithmetic on the BF16
 * weights.  set_weights copies host weights and resets the Adam state;
 * get_weights returns the masters (host). */
int dgidp_mlp_set_weights(dgidp_ctx* ctx, const float* w);
int dgidp_mlp_get_weights(dgidp_ctx* ctx, float* w);
/* y[B] = network(x[B][16]), 0 <= B <= 2^30.  Device inputs (on_device) must be
 * 16-byte aligned, else DGIDP_E_INVALID_ARG. */
int dgidp_mlp_forward(dgidp_ctx* ctx, const float* x, int64_t B, float* y, int on_device);
/* Gradient of loss = (1/B) sum_s (y_s - t_s)^2 at the BF16 weights, into
 * grad[DGIDP_MLP_NPARAM] (host or device as on_device); *loss (host, may be
 * NULL) receives the loss.  Deterministic. */
int dgidp_mlp_grad(dgidp_ctx* ctx, const float* x, const float* t, int64_t B, float* grad, float* loss,
                   int on_device);
/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, learning rate lr > 0) on
 * that gradient, applied to the FP32 masters; new BF16 copy.  *loss (host,
 * may be NULL) receives the loss before the step. */
int dgidp_mlp_train_step(dgidp_ctx* ctx, const float* x, const float* t, int64_t B, float lr,
                         float* loss, int on_device);

/* Mean duration in milliseconds of one launch of each kernel of a step,
 * measured with HIP events on the context's stream over back-to-back launches:
 * ms[0] the element stage kernel, averaged over `reps` rounds of its three
 * SSP-RK3 stage configurations (stage 1 reads one state, stages 2 and 3 read
 * two), ms[1] the mortar limiter kernel, ms[2] the time-step reduction.
 * Uses the current state; leaves it unchanged (outputs go to scratch
 * buffers).  Synchronises. */
int dgidp_time_kernels(dgidp_ctx* ctx, int reps, double* ms);

/* Host-only: the operator tables the library uploads for degree N, flat
 * doubles: w[n] (LGL weights, Sec. 2.1), Sbar[n][n] (Sec. 2.1), mortar
 * interpolation I[2][n][n] and L2 projection P[2][n][n] (Sec. 2.2, Kopriva's
 * mortar), sparse mortar weights Wt[n][2n] (eq. local_weights, App. A), and the
 * nodal-to-modal transform Vinv[n][n] onto orthonormal Legendre polynomials
 * (indicator and features); n = N+1.  `out` holds at least n + 8 n^2 doubles.
 * Needs no GPU. */
int dgidp_host_tables(int N, double* out);

#ifdef __cplusplus
}
#endif

#endif
