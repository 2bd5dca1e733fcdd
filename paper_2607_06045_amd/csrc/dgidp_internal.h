// Internal declarations shared by the host code and the HIP kernels of dgidp.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/dgidp.h"

namespace dgidp {

constexpr int kMaxN = 4;
constexpr int kSlotW = 16;  // doubles per mortar slot record
// elements per block of the stage kernel (the host orders elements per the
// kernel's block-to-XCD mapping)
constexpr int stage_block_elems(int N) { return N == 3 ? 4 : 5; }

// Face codes: fmort[e*4+f] = -1 for a conforming face, otherwise
// (mortar << 2) | (small << 1) | half, small = 1 if e is a small side.
inline __host__ __device__ int fm_mortar(int c) { return c >> 2; }
inline __host__ __device__ int fm_small(int c) { return (c >> 1) & 1; }
inline __host__ __device__ int fm_half(int c) { return c & 1; }

// Operator tables of degree N, in constant memory.
template <int N>
struct Tab {
    static constexpr int n = N + 1;
    double w[n];                  // LGL quadrature weights
    double winv[n];               // 1 / w
    double S[n][n];               // Sbar = 2 Qbar - Bbar
    double I[2][n][n];            // mortar interpolation: half h, small node l, large node k
    double P[2][n][n];            // L2 projection: half h, large node k, small node l
    double Wt[n][2 * n];          // sparse mortar weights, reference measure on [-1, 1]
    // their nonzero entries: per large-face node k the count and the columns
    // h n + l in ascending order; per small-face node (h, l) the count and the
    // large-face nodes k in ascending order
    int lnc[n], lnz[n][2 * n];
    int snc[2][n], snz[2][n][n];
    float wf[n], Sf[n][n], If[2][n][n], Pf[2][n][n];  // FP32 copies for the mixed mode
    double Vinv[n][n];            // nodal -> modal, orthonormal Legendre: m_i = sum_a Vinv[i][a] q_a
};

// Device-side statistics accumulator.
struct DevStats {
    unsigned long long fv_inadmissible;
    unsigned long long violations;
    unsigned long long theta_vol_min_bits;   // min over positive doubles as bit patterns
    unsigned long long theta_mort_min_bits;
    double alpha_vol_sum;
    double alpha_mort_sum;
    unsigned long long nfaces;
    unsigned long long nmortars;
    double dt;
};

struct DevMesh {
    int E = 0, M = 0;
    int* fnbr = nullptr;        // [E*4] neighbour element across the face (large element for small sides)
    int* fnbr2 = nullptr;       // [E*4] second small element across a large face, else -1
    int* fmort = nullptr;       // [E*4] face codes
    int* mort = nullptr;        // [M*4] large element, large face, small 0, small 1
    double* h = nullptr;        // [E*2] hx, hy
    int* slot_node = nullptr;   // [M*3n] element * n^2 + node
    int* slot_partner = nullptr;  // [M*3n] slot of the other mortar of a node on two mortars, or -1
    double* slot = nullptr;     // [M*3n*kSlotW]
    int* perm = nullptr;        // [E] external index of internal element e
    double* shock_ind = nullptr;  // [E] shock indicator of combined limiting (internal order)
    double* dlo = nullptr;      // [E*4*NN] R_LO / m of a stage's input (low-order-solution bounds)
    double* lob = nullptr;      // [E*3*NN] rho min, rho max, ln s min from the low-order solution
    double* lsv = nullptr;      // [E*2*NN] low-order density and ln s per node
    // [ceil(E / stage_block_elems(N))] stage-kernel element batches: the nbm
    // batches holding an element with a mortar face first, then the others,
    // each part in ascending order
    int* blist = nullptr;
    int nbm = 0;
    int8_t* bkind = nullptr;    // [NB] condition of each boundary node (external numbering)
    double* bext = nullptr;     // [NB*4] exterior state of each boundary node
};

struct KernelParams {
    double gamma, beta;
    int limiter;
    int precision;
    int vflux;
};

// the dt maximum is merged into kDtSpread accumulators kDtStride words apart
// (one cache line each), so that the per-block atomics do not all meet at one
// address; an accumulator set holds kDtSpread * kDtStride words
constexpr int kDtSpread = 64;
constexpr int kDtStride = 16;
constexpr int kDtWords = kDtSpread * kDtStride;

// where a stage kernel takes dt from: a stored value (dt), or the maximum that
// the dt kernel accumulated (dtmax, then dt = cfl / max, stored to dt_out)
struct DtSource {
    const double* dt = nullptr;
    const unsigned long long* dtmax = nullptr;
    double cfl = 0.0;
    double* dt_out = nullptr;
};

// new leaf list of an adaptation and its source map (external leaf ids):
// kind 0 kept (src[0] the old leaf), 1 child (src[0] the old parent, src[1] the
// child index cx + 2 cy), 2 parent (src[0..3] the old children by child index)
struct AdaptPlan {
    std::vector<int8_t> level;
    std::vector<int32_t> ix, iy;
    std::vector<int8_t> kind;
    std::vector<int64_t> src;  // [4 * new leaves]
    int64_t n_refined = 0, n_balance = 0, n_coarsened = 0;
};
int adapt_leaves(int64_t E, const int8_t* lev, const int32_t* ix, const int32_t* iy, int nx0,
                 int ny0, const int8_t* flags, AdaptPlan& plan, std::string& err);

// transfer onto a new mesh, new internal element order: tkind[e] 0 copy,
// 1 child, 2 parent; tsrc[e][4] old internal elements (child: parent, child
// index).  Zhang-Shu groups zgrp[g][6] = kind (1 refine, 2 coarsen), old
// parent (refine), new elements (4 children, or the parent and -1).
int launch_transfer(int N, int E_new, const int* tkind, const int* tsrc, const double* uold,
                    double* unew, hipStream_t s);
int launch_zhang_shu(int N, int G, const int* zgrp, const double* uold, double* unew, double eps,
                     double gamma, unsigned long long* counts, hipStream_t s);

// modal indicator alpha[E] and features feat[E][16], external order (either may be null)
int launch_indicator(int N, int E, const double* u, const int* perm, double gamma, float* alpha,
                     float* feat, hipStream_t s);
// learned indicator alpha[E] (external order): features and network in one kernel;
// wb the network's BF16 parameters
int launch_learned_indicator(int N, int E, const double* u, const int* perm, double gamma, const uint16_t* wb,
                             float* alpha, hipStream_t s);

// learned indicator network (dgidp_mlp.hip); device pointers on stream st
struct MlpState;
int mlp_num_params();
MlpState* mlp_create();
void mlp_destroy(MlpState* s);
bool mlp_has_weights(const MlpState* s);
float* mlp_scratch(MlpState* s, int which, size_t floats);  // which in 0..3, grown on demand
int mlp_set_weights(MlpState* s, const float* host_w, hipStream_t st);
int mlp_get_weights(MlpState* s, float* host_w, hipStream_t st);
const uint16_t* mlp_weights_bf16(const MlpState* s);  // device, DGIDP_MLP_NPARAM values and a zero tail to 5,320
int mlp_forward(MlpState* s, const float* x, int64_t B, float* y, hipStream_t st);
// gradient (to grad, if not null) and loss (to *loss_host, if not null); an
// Adam step when lr > 0
int mlp_grad_step(MlpState* s, const float* x, const float* t, int64_t B, float lr, float* grad,
                  float* loss_host, hipStream_t st);

// launchers (dgidp_kernels.hip)
// rev: the conforming launch of a split stage walks each XCD's batch range from
// its end (the middle stage of SSP-RK3, so that every stage starts where the
// kernel before it finished writing its input)
int launch_stage(int N, const DevMesh& m, const KernelParams& kp, const double* uin,
                 const double* un, double* uout, double a, double b, const DtSource& dt,
                 DevStats* st, hipStream_t s, bool rev = false);
int launch_rhs(int N, const DevMesh& m, const KernelParams& kp, const double* u, int which,
               double* du, hipStream_t s);
int launch_mortar(int N, const DevMesh& m, double* uout, double b, DevStats* st, hipStream_t s,
                  double gamma, int limiter);
// per-element shock indicator on the pressure of u into m.shock_ind (combined limiting)
int launch_shock_indicator(int N, const DevMesh& m, const double* u, double gamma, hipStream_t s);
// local bounds from the low-order solution u + dt * dlo into lob (eq. Bounds_LowOrder);
// lsv [E*2*NN] holds the per-node low-order density and log entropy between the passes
int launch_lowbounds(int N, const DevMesh& m, double gamma, const double* u, const double* dlo,
                     const DtSource& dt, double* lsv, double* lob, hipStream_t s);
// max over nodes of the dt denominator, atomically merged into the accumulator
// set acc (all zero on entry); the set other is cleared for the next step
int launch_dt(int N, const DevMesh& m, const KernelParams& kp, const double* u, int mode,
              unsigned long long* acc, unsigned long long* other, hipStream_t s);
int launch_permute(int N, int E, const int* perm, const double* src, double* dst, int to_internal,
                   hipStream_t s);
int launch_stats_reset(DevStats* st, hipStream_t s);
int launch_set_double(double* p, double v, hipStream_t s);
int launch_check_state(int N, int E, double gamma, const double* u, unsigned long long* bad,
                       hipStream_t s);
int upload_tables(int N, const void* host_tab, size_t bytes);

// allocation-free step (dgidp_noalloc.hip): the size of the static per-device
// scratch array, its one-time set-up on the current device (hipGetSymbolAddress;
// 0 on success), its device address on the current device (null if not set up),
// and a fill kernel for clearing parts of it
constexpr size_t kNoallocScratchBytes = size_t(64) << 20;
int noalloc_scratch_setup();
void* noalloc_scratch(size_t* bytes);
int launch_fill_u64(unsigned long long* p, int n, unsigned long long v, hipStream_t s);

}  // namespace dgidp
