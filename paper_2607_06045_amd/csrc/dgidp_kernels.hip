// HIP kernels of dgidp for gfx950 (MI355X).
//
// One SSP-RK3 stage (Sec. 2.3 and Sec. 3 intro of the paper) is two kernels:
//   k_stage   one thread per LGL node, a block holds 256 / (N+1)^2 elements.
//             Loads the element into LDS, evaluates the Ranocha two-point
//             fluxes once per node pair of every line, telescopes them into
//             high-order subcell fluxes (eq. fluxdifferencingform), evaluates the
//             LLF subcell fluxes (eq. FVmethod), the conforming surface fluxes and
//             this element's side of every mortar (Kopriva's L2 mortar and the
//             sparse IDP mortar flux of eq. interfaceflux_local), forms the
//             low-order update and the positivity bounds (eq. Bounds_Positivity),
//             limits the volume antidiffusive fluxes per subcell face and writes
//             a u^n + b u^vol.  Nodes on mortars also leave a slot record with
//             their mortar antidiffusive increment and their own admissible
//             fraction of it.
//   k_mortar  one thread per mortar slot: the mortar's factor is the minimum
//             over its slots (one factor per mortar keeps the flux conservative,
//             Sec. 2.3); the corrections are added in ascending mortar order.
// The time step (eq. timestep_restriction) is a grid max-reduction, k_dt.
#include <hip/hip_runtime.h>

#include "dgidp_internal.h"

namespace dgidp {

__constant__ Tab<3> c_tab3;
__constant__ Tab<4> c_tab4;

template <int N>
__device__ __forceinline__ const Tab<N>& T();
template <>
__device__ __forceinline__ const Tab<3>& T<3>() { return c_tab3; }
template <>
__device__ __forceinline__ const Tab<4>& T<4>() { return c_tab4; }

int upload_tables(int N, const void* host_tab, size_t bytes)
{
    hipError_t e = hipErrorInvalidValue;
    if (N == 3 && bytes == sizeof(Tab<3>)) e = hipMemcpyToSymbol(HIP_SYMBOL(c_tab3), host_tab, bytes);
    if (N == 4 && bytes == sizeof(Tab<4>)) e = hipMemcpyToSymbol(HIP_SYMBOL(c_tab4), host_tab, bytes);
    return e == hipSuccess ? 0 : -1;
}

// Workgroups are dispatched round-robin over the 8 XCDs; give each XCD a
// contiguous range of element batches so that face neighbours share its L2.
__device__ __forceinline__ int xcd_batch(int bid, int nb)
{
    const int q = nb >> 3, r = nb & 7;
    const int x = bid & 7, j = bid >> 3;
    return (x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q) + j;
}

// ---------------------------------------------------------------------------
// Euler helpers
// ---------------------------------------------------------------------------
struct NodeP {
    double u[4];
    double r, v1, v2, p, c;
};

__device__ __forceinline__ void make_node(NodeP& s, double g)
{
    const double ir = 1.0 / s.u[0];
    s.r = s.u[0];
    s.v1 = s.u[1] * ir;
    s.v2 = s.u[2] * ir;
    s.p = (g - 1.0) * (s.u[3] - 0.5 * (s.u[1] * s.v1 + s.u[2] * s.v2));
    s.c = sqrt(g * s.p * ir);
}

__device__ __forceinline__ double pressure(const double* u, double g)
{
    return (g - 1.0) * (u[3] - 0.5 * (u[1] * u[1] + u[2] * u[2]) / u[0]);
}

// local Lax-Friedrichs flux in direction d between the low-side state L and the
// high-side state R
template <int D>
__device__ __forceinline__ void llf(const NodeP& L, const NodeP& R, double* F)
{
    const double vL = D == 0 ? L.v1 : L.v2, vR = D == 0 ? R.v1 : R.v2;
    const double lam = fmax(fabs(vL) + L.c, fabs(vR) + R.c);
    double fL[4], fR[4];
    fL[0] = L.r * vL;
    fL[1] = L.u[1] * vL + (D == 0 ? L.p : 0.0);
    fL[2] = L.u[2] * vL + (D == 1 ? L.p : 0.0);
    fL[3] = (L.u[3] + L.p) * vL;
    fR[0] = R.r * vR;
    fR[1] = R.u[1] * vR + (D == 0 ? R.p : 0.0);
    fR[2] = R.u[2] * vR + (D == 1 ? R.p : 0.0);
    fR[3] = (R.u[3] + R.p) * vR;
#pragma unroll
    for (int v = 0; v < 4; ++v) F[v] = 0.5 * (fL[v] + fR[v]) - 0.5 * lam * (R.u[v] - L.u[v]);
}

__device__ __forceinline__ void llf_dir(int d, const NodeP& L, const NodeP& R, double* F)
{
    if (d == 0) llf<0>(L, R, F);
    else llf<1>(L, R, F);
}

// LLF flux on a mortar node between the interpolated large-face state ui and
// the small-face state us.  An interpolated state outside the admissible set
// leaves the high-order mortar flux undefined (NaN); the mortar limiter then
// keeps the low-order flux for the whole mortar.
__device__ __forceinline__ void mortar_flux(int d, bool large_low, const NodeP& ui, const NodeP& us,
                                            double* F)
{
    if (!(ui.r > 0.0) || !(ui.p > 0.0)) {
        const double nan = __builtin_nan("");
        F[0] = F[1] = F[2] = F[3] = nan;
        return;
    }
    if (large_low) llf_dir(d, ui, us, F);
    else llf_dir(d, us, ui, F);
}

// logarithmic mean (x - y) / (ln x - ln y) from precomputed logarithms; for
// ((x-y)/(x+y))^2 < 1e-4 the truncated series of 2 atanh (Ismail & Roe 2009)
__device__ __forceinline__ double lnmean(double x, double y, double lx, double ly)
{
    const double s = x + y, d = x - y;
    if (d * d < 1e-4 * (s * s)) {
        const double f2 = (d * d) / (s * s);
        return s / (2.0 + f2 * (2.0 / 3.0 + f2 * (2.0 / 5.0 + f2 * (2.0 / 7.0))));
    }
    return d / (lx - ly);
}

__device__ __forceinline__ float lnmeanf(float x, float y, float lx, float ly)
{
    const float s = x + y, d = x - y;
    if (d * d < 1e-2f * (s * s)) {
        const float f2 = (d * d) / (s * s);
        return s / (2.0f + f2 * (2.0f / 3.0f + f2 * (2.0f / 5.0f + f2 * (2.0f / 7.0f))));
    }
    return d / (lx - ly);
}

// ---------------------------------------------------------------------------
// pressure blending factor: largest theta in [0,1] with rho(u0 + theta dc) > 0
// and p(u0 + theta dc) >= pt.  For rho > 0, p >= pt is
// g(theta) = (E - pt/(gamma-1)) rho - |m|^2 / 2 >= 0, a quadratic in theta whose
// admissible set along the ray is an interval [0, theta*] (p is concave).
// ---------------------------------------------------------------------------
__device__ __forceinline__ double theta_p(const double* u0, const double* dc, double pt, double g)
{
    const double e0 = u0[3] - pt / (g - 1.0);
    const double g0 = u0[0] * e0 - 0.5 * (u0[1] * u0[1] + u0[2] * u0[2]);
    if (!(g0 > 0.0) || !(u0[0] > 0.0)) return 0.0;
    // full step admissible: the interval contains [0, 1]
    const double r1 = u0[0] + dc[0];
    if (r1 > 0.0) {
        const double m1 = u0[1] + dc[1], m2 = u0[2] + dc[2];
        const double g1v = (u0[3] + dc[3] - pt / (g - 1.0)) * r1 - 0.5 * (m1 * m1 + m2 * m2);
        if (g1v >= 0.0) return 1.0;
    }
    const double g1 = dc[0] * e0 + u0[0] * dc[3] - (u0[1] * dc[1] + u0[2] * dc[2]);
    const double g2 = dc[0] * dc[3] - 0.5 * (dc[1] * dc[1] + dc[2] * dc[2]);
    double root = 1.0;
    if (g2 == 0.0) {
        if (g1 < 0.0) root = fmin(root, -g0 / g1);
    } else {
        const double disc = g1 * g1 - 4.0 * g2 * g0;
        if (disc >= 0.0) {
            const double sq = sqrt(disc);
            const double qq = -0.5 * (g1 + (g1 >= 0.0 ? sq : -sq));
            const double ra = qq / g2, rb = g0 / qq;
            if (ra > 0.0) root = fmin(root, ra);
            if (rb > 0.0) root = fmin(root, rb);
        }
    }
    if (dc[0] < 0.0) root = fmin(root, -u0[0] / dc[0]);
    return root;
}

// the limiter aims at the bounds raised by this relative margin so that the
// rounding of the final sums cannot cross the bounds themselves
constexpr double kMargin = 1.0 + 0x1p-40;

// ---------------------------------------------------------------------------
// statistics
// ---------------------------------------------------------------------------
template <typename TT>
__device__ __forceinline__ TT wave_sum(TT v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ double wave_min(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
    return v;
}

__device__ __forceinline__ double wave_max(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

// block-wide accumulation of per-thread statistics, one atomic per wave
__device__ __forceinline__ void push_stats(DevStats* st, unsigned long long inad,
                                           unsigned long long viol, double thmin, double asum,
                                           unsigned long long nf, bool mortar)
{
    inad = wave_sum(inad);
    viol = wave_sum(viol);
    asum = wave_sum(asum);
    nf = wave_sum(nf);
    thmin = wave_min(thmin);
    if ((threadIdx.x & 63) == 0) {
        if (inad) atomicAdd(&st->fv_inadmissible, inad);
        if (viol) atomicAdd(&st->violations, viol);
        if (nf) {
            if (mortar) {
                atomicAdd(&st->alpha_mort_sum, asum);
                atomicAdd(&st->nmortars, nf);
            } else {
                atomicAdd(&st->alpha_vol_sum, asum);
                atomicAdd(&st->nfaces, nf);
            }
        }
        if (thmin < 1.0) {
            unsigned long long bits = __double_as_longlong(fmax(thmin, 0.0));
            atomicMin(mortar ? &st->theta_mort_min_bits : &st->theta_vol_min_bits, bits);
        }
    }
}

// ---------------------------------------------------------------------------
// element kernel
// ---------------------------------------------------------------------------
enum { MODE_STAGE = 0, MODE_RHS_HIGH = 1, MODE_RHS_LOW = 2 };

struct StageArgs {
    const double* uin;
    const double* un;
    double* uout;
    double a, b;
    const double* dt;
    const int* fnbr;
    const int* fmort;
    const int* mort;
    const double* h;
    double* slot;
    int E;
    double gamma, beta;
    int limiter;
    DevStats* st;
};

// node (a, b) at position k along face f
template <int N>
__device__ __forceinline__ int face_q(int f, int k)
{
    constexpr int n = N + 1;
    return f == 0 ? k * n : (f == 1 ? k * n + N : (f == 2 ? k : N * n + k));
}

template <int N>
__device__ __forceinline__ void load_node(const double* u, int e, int q, NodeP& s, double g)
{
    constexpr int NN = (N + 1) * (N + 1);
#pragma unroll
    for (int v = 0; v < 4; ++v) s.u[v] = u[((size_t)e * 4 + v) * NN + q];
    make_node(s, g);
}

// pair (l, k), l < k, number i of a line
template <int N>
__device__ __forceinline__ void pair_lk(int i, int& l, int& k)
{
    constexpr int n = N + 1;
    int r = i;
    l = 0;
    while (r >= n - 1 - l) {
        r -= n - 1 - l;
        ++l;
    }
    k = l + 1 + r;
}

template <int N, int MODE, bool MIXED>
__global__ __launch_bounds__(256) void k_stage(StageArgs A)
{
    constexpr int n = N + 1, NN = n * n, EPB = 256 / NN, NT = EPB * NN;
    constexpr int NPL = n * (n - 1) / 2;   // node pairs per line
    constexpr int NP = 2 * n * NPL;        // node pairs per element
    constexpr int NF = 2 * N * n;          // interior subcell faces per element
    constexpr int PPT = NP / NN;           // pairs per thread (3 for N=3, 4 for N=4)
    static_assert(NP % NN == 0, "pair split");
    static_assert(NP >= 2 * NF, "face buffers reuse the pair buffer");
    static_assert(NP * 4 >= 4 * 2 * n * 4, "mortar node fluxes reuse the pair buffer");

    __shared__ double sU[EPB][4][NN];
    __shared__ double sR[EPB][7][NN];  // rho, v1, v2, p, c, ln rho, ln(rho/p)
    __shared__ double sPair[EPB][NP * 4];
    __shared__ double sTh[EPB][NN];

    const Tab<N>& tb = T<N>();
    const double g = A.gamma;
    const int tid = threadIdx.x;
    const int le = tid / NN, q = tid - le * NN, a = q % n, b = q / n;
    const int e = xcd_batch(blockIdx.x, gridDim.x) * EPB + le;
    const bool act = tid < NT && e < A.E;

    NodeP me;
    double hx = 1.0, hy = 1.0;
    int fcode[4] = {-1, -1, -1, -1}, fn[4] = {0, 0, 0, 0};
    if (act) {
        load_node<N>(A.uin, e, q, me, g);
        hx = A.h[2 * e];
        hy = A.h[2 * e + 1];
#pragma unroll
        for (int v = 0; v < 4; ++v) sU[le][v][q] = me.u[v];
        sR[le][0][q] = me.r;
        sR[le][1][q] = me.v1;
        sR[le][2][q] = me.v2;
        sR[le][3][q] = me.p;
        sR[le][4][q] = me.c;
        sR[le][5][q] = log(me.r);
        sR[le][6][q] = log(me.r / me.p);
#pragma unroll
        for (int f = 0; f < 4; ++f) {
            fcode[f] = A.fmort[e * 4 + f];
            fn[f] = A.fnbr[e * 4 + f];
        }
    }
    // faces this node lies on: position along the face
    const int kpos[4] = {b, b, a, a};
    const bool onf[4] = {a == 0, a == N, b == 0, b == N};
    __syncthreads();

    // ---- phase 2: mortar-node fluxes of large faces (Kopriva's L2 mortar) ----
    if (act) {
#pragma unroll
        for (int f = 0; f < 4; ++f) {
            if (!onf[f] || fcode[f] < 0 || fm_small(fcode[f])) continue;
            const int S = fm_mortar(fcode[f]), k = kpos[f], d = f >> 1;
            const bool large_low = f & 1;
            for (int hh = 0; hh < 2; ++hh) {
                const int s = A.mort[S * 4 + 2 + hh];
                NodeP ui, us;
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    double acc = 0.0;
#pragma unroll
                    for (int j = 0; j < n; ++j) acc += tb.I[hh][k][j] * sU[le][v][face_q<N>(f, j)];
                    ui.u[v] = acc;
                }
                make_node(ui, g);
                load_node<N>(A.uin, s, face_q<N>(f ^ 1, k), us, g);
                double F[4];
                mortar_flux(d, large_low, ui, us, F);
#pragma unroll
                for (int v = 0; v < 4; ++v) sPair[le][((f * 2 + hh) * n + k) * 4 + v] = F[v];
            }
        }
    }
    __syncthreads();

    // ---- phase 3: surface contributions of this node ----
    double RsLO[4] = {0, 0, 0, 0};
    double dS[2][4] = {{0, 0, 0, 0}, {0, 0, 0, 0}};  // HO - LO of up to two mortar faces
    int slotid[2] = {-1, -1};
    int nmf = 0;
    if (act) {
#pragma unroll
        for (int f = 0; f < 4; ++f) {
            if (!onf[f]) continue;
            const int k = kpos[f], d = f >> 1;
            const double hf = f < 2 ? hy : hx;
            const bool low = f & 1;  // this element lies on the low side of the face
            const double sg = low ? -1.0 : 1.0;
            const int code = fcode[f];
            if (code < 0) {
                NodeP o;
                load_node<N>(A.uin, fn[f], face_q<N>(f ^ 1, k), o, g);
                double F[4];
                if (low) llf_dir(d, me, o, F);
                else llf_dir(d, o, me, F);
                const double W = sg * tb.w[k] * hf * 0.5;
#pragma unroll
                for (int v = 0; v < 4; ++v) RsLO[v] += W * F[v];
                continue;
            }
            const int S = fm_mortar(code);
            double ho[4] = {0, 0, 0, 0}, lo[4] = {0, 0, 0, 0};
            if (!fm_small(code)) {
                // large side: project the mortar fluxes, sparse low-order pairs
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    double acc = 0.0;
#pragma unroll
                    for (int hh = 0; hh < 2; ++hh)
#pragma unroll
                        for (int l = 0; l < n; ++l)
                            acc += tb.P[hh][k][l] * sPair[le][((f * 2 + hh) * n + l) * 4 + v];
                    ho[v] = sg * tb.w[k] * hf * 0.5 * acc;
                }
                for (int hh = 0; hh < 2; ++hh) {
                    const int s = A.mort[S * 4 + 2 + hh];
                    for (int l = 0; l < n; ++l) {
                        const double wt = tb.Wt[k][hh * n + l];
                        if (wt == 0.0) continue;
                        NodeP us;
                        load_node<N>(A.uin, s, face_q<N>(f ^ 1, l), us, g);
                        double G[4];
                        if (low) llf_dir(d, me, us, G);
                        else llf_dir(d, us, me, G);
                        const double W = sg * wt * hf * 0.5;
#pragma unroll
                        for (int v = 0; v < 4; ++v) lo[v] += W * G[v];
                    }
                }
                slotid[nmf] = S * 3 * n + k;
            } else {
                // small side: interpolate the large face, LLF on the mortar = this face
                const int hh = fm_half(code), L = fn[f], fl = f ^ 1;
                const double hL = 2.0 * hf;
                NodeP uL[n];
#pragma unroll
                for (int j = 0; j < n; ++j) load_node<N>(A.uin, L, face_q<N>(fl, j), uL[j], g);
                NodeP ui;
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    double acc = 0.0;
#pragma unroll
                    for (int j = 0; j < n; ++j) acc += tb.I[hh][k][j] * uL[j].u[v];
                    ui.u[v] = acc;
                }
                make_node(ui, g);
                double F[4];
                mortar_flux(d, !low, ui, me, F);
#pragma unroll
                for (int v = 0; v < 4; ++v) ho[v] = sg * tb.w[k] * hf * 0.5 * F[v];
#pragma unroll
                for (int j = 0; j < n; ++j) {
                    const double wt = tb.Wt[j][hh * n + k];
                    if (wt == 0.0) continue;
                    double G[4];
                    if (low) llf_dir(d, me, uL[j], G);
                    else llf_dir(d, uL[j], me, G);
                    const double W = sg * wt * hL * 0.5;
#pragma unroll
                    for (int v = 0; v < 4; ++v) lo[v] += W * G[v];
                }
                slotid[nmf] = S * 3 * n + n + hh * n + k;
            }
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                RsLO[v] += lo[v];
                dS[nmf][v] = ho[v] - lo[v];
            }
            ++nmf;
        }
    }
    __syncthreads();

    // ---- phase 4: two-point volume fluxes, once per node pair of each line ----
    if (act) {
#pragma unroll
        for (int i = 0; i < PPT; ++i) {
            const int p = q + i * NN;
            const int d = p / (n * NPL), rem = p - d * (n * NPL);
            const int line = rem / NPL, pi = rem - line * NPL;
            int l, k;
            pair_lk<N>(pi, l, k);
            const int ql = d == 0 ? line * n + l : l * n + line;
            const int qk = d == 0 ? line * n + k : k * n + line;
            const double scale = tb.S[l][k] * 0.5 * (d == 0 ? hy : hx);
            double f[4];
            if (!MIXED) {
                const double rL = sR[le][0][ql], rR = sR[le][0][qk];
                const double v1L = sR[le][1][ql], v1R = sR[le][1][qk];
                const double v2L = sR[le][2][ql], v2R = sR[le][2][qk];
                const double pL = sR[le][3][ql], pR = sR[le][3][qk];
                const double rho_ln = lnmean(rL, rR, sR[le][5][ql], sR[le][5][qk]);
                const double zL = rL / pL, zR = rR / pR;
                const double z_ln = lnmean(zL, zR, sR[le][6][ql], sR[le][6][qk]);
                const double vnL = d == 0 ? v1L : v2L, vnR = d == 0 ? v1R : v2R;
                const double fr = rho_ln * 0.5 * (vnL + vnR);
                const double pa = 0.5 * (pL + pR);
                f[0] = fr;
                f[1] = fr * 0.5 * (v1L + v1R) + (d == 0 ? pa : 0.0);
                f[2] = fr * 0.5 * (v2L + v2R) + (d == 1 ? pa : 0.0);
                f[3] = fr * (0.5 * (v1L * v1R + v2L * v2R) + 1.0 / ((g - 1.0) * z_ln)) +
                       0.5 * (pL * vnR + pR * vnL);
            } else {
                const float rL = (float)sR[le][0][ql], rR = (float)sR[le][0][qk];
                const float v1L = (float)sR[le][1][ql], v1R = (float)sR[le][1][qk];
                const float v2L = (float)sR[le][2][ql], v2R = (float)sR[le][2][qk];
                const float pL = (float)sR[le][3][ql], pR = (float)sR[le][3][qk];
                const float rho_ln = lnmeanf(rL, rR, (float)sR[le][5][ql], (float)sR[le][5][qk]);
                const float zL = rL / pL, zR = rR / pR;
                const float z_ln = lnmeanf(zL, zR, (float)sR[le][6][ql], (float)sR[le][6][qk]);
                const float vnL = d == 0 ? v1L : v2L, vnR = d == 0 ? v1R : v2R;
                const float fr = rho_ln * 0.5f * (vnL + vnR);
                const float pa = 0.5f * (pL + pR);
                f[0] = fr;
                f[1] = fr * 0.5f * (v1L + v1R) + (d == 0 ? pa : 0.0f);
                f[2] = fr * 0.5f * (v2L + v2R) + (d == 1 ? pa : 0.0f);
                f[3] = fr * (0.5f * (v1L * v1R + v2L * v2R) + 1.0f / ((float)(g - 1.0) * z_ln)) +
                       0.5f * (pL * vnR + pR * vnL);
            }
#pragma unroll
            for (int v = 0; v < 4; ++v) sPair[le][p * 4 + v] = scale * f[v];
        }
    }
    __syncthreads();

    // ---- phase 5: subcell faces owned by this node: x (a|a+1) and y (b|b+1) ----
    double FVo[2][4], Ao[2][4];
    if (act) {
#pragma unroll
        for (int d = 0; d < 2; ++d) {
            const int pos = d == 0 ? a : b, line = d == 0 ? b : a;
            if (pos >= N) continue;
            double ho[4] = {0, 0, 0, 0};
            // telescoped high-order flux: pairs (l, k) with l <= pos < k
#pragma unroll
            for (int l = 0; l <= pos; ++l)
#pragma unroll
                for (int k = pos + 1; k < n; ++k) {
                    const int pi = l * (2 * n - l - 1) / 2 + (k - l - 1);
                    const int p = d * n * NPL + line * NPL + pi;
#pragma unroll
                    for (int v = 0; v < 4; ++v) ho[v] += sPair[le][p * 4 + v];
                }
            const int qn = d == 0 ? q + 1 : q + n;
            NodeP o;
#pragma unroll
            for (int v = 0; v < 4; ++v) o.u[v] = sU[le][v][qn];
            o.r = sR[le][0][qn];
            o.v1 = sR[le][1][qn];
            o.v2 = sR[le][2][qn];
            o.p = sR[le][3][qn];
            o.c = sR[le][4][qn];
            double F[4];
            llf_dir(d, me, o, F);
            const double hs = 0.5 * (d == 0 ? hy : hx), wl = tb.w[line];
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                FVo[d][v] = hs * F[v];
                Ao[d][v] = wl * (ho[v] - FVo[d][v]);
            }
        }
    }
    __syncthreads();
    double* sFV = sPair[le];
    double* sA = sPair[le] + NF * 4;
    if (act) {
        if (a < N) {
            const int fi = b * N + a;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                sFV[fi * 4 + v] = FVo[0][v];
                sA[fi * 4 + v] = Ao[0][v];
            }
        }
        if (b < N) {
            const int fi = N * n + a * N + b;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                sFV[fi * 4 + v] = FVo[1][v];
                sA[fi * 4 + v] = Ao[1][v];
            }
        }
    }
    __syncthreads();

    // ---- phase 6: low-order residual, bounds, node factors ----
    const int fxl = b * N + a - 1, fxr = b * N + a;          // x faces left / right of the node
    const int fyb = N * n + a * N + b - 1, fyt = N * n + a * N + b;  // y faces below / above
    double RLO[4];
    double mi = 1.0;
    if (act) {
        mi = 0.25 * hx * hy * tb.w[a] * tb.w[b];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            double r = RsLO[v];
            if (a > 0) r += tb.w[b] * sFV[fxl * 4 + v];
            if (a < N) r -= tb.w[b] * sFV[fxr * 4 + v];
            if (b > 0) r += tb.w[a] * sFV[fyb * 4 + v];
            if (b < N) r -= tb.w[a] * sFV[fyt * 4 + v];
            RLO[v] = r;
        }
    }
    if (MODE == MODE_RHS_LOW || MODE == MODE_RHS_HIGH) {
        if (act) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                double r = RLO[v];
                if (MODE == MODE_RHS_HIGH) {
                    if (a > 0) r += sA[fxl * 4 + v];
                    if (a < N) r -= sA[fxr * 4 + v];
                    if (b > 0) r += sA[fyb * 4 + v];
                    if (b < N) r -= sA[fyt * 4 + v];
                    r += dS[0][v] + dS[1][v];
                }
                A.uout[((size_t)e * 4 + v) * NN + q] = r / mi;
            }
        }
        return;
    }

    const double dt = *A.dt;
    const double dtm = dt / mi;
    double uFV[4], cf[4][4];
    double rmin = 0.0, pmin = 0.0, th = 1.0;
    unsigned long long inad = 0;
    if (act) {
#pragma unroll
        for (int v = 0; v < 4; ++v) uFV[v] = me.u[v] + dtm * RLO[v];
        const double pFV = pressure(uFV, g);
        if (!(uFV[0] > 0.0) || !(pFV > 0.0)) inad = 1;
        rmin = A.beta * uFV[0];
        pmin = A.beta * pFV;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            cf[0][v] = a > 0 ? dtm * sA[fxl * 4 + v] : 0.0;
            cf[1][v] = a < N ? -dtm * sA[fxr * 4 + v] : 0.0;
            cf[2][v] = b > 0 ? dtm * sA[fyb * 4 + v] : 0.0;
            cf[3][v] = b < N ? -dtm * sA[fyt * 4 + v] : 0.0;
        }
        if (A.limiter != DGIDP_LIMIT_NONE) {
            // Zalesak-type factor for the density: sum of the negative increments
            const double rt = rmin * kMargin, pt = pmin * kMargin;
            double P = 0.0;
#pragma unroll
            for (int j = 0; j < 4; ++j) P += fmin(cf[j][0], 0.0);
            if (P < 0.0) th = fmax(fmin((rt - uFV[0]) / P, 1.0), 0.0);
            // pressure: each face's increment scaled by Gamma = 2d = 4
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const double dc[4] = {4.0 * cf[j][0], 4.0 * cf[j][1], 4.0 * cf[j][2], 4.0 * cf[j][3]};
                if (dc[0] == 0.0 && dc[1] == 0.0 && dc[2] == 0.0 && dc[3] == 0.0) continue;
                th = fmin(th, theta_p(uFV, dc, pt, g));
            }
        }
        sTh[le][q] = th;
    }
    __syncthreads();

    // ---- phase 7: limited volume update, SSP combination, mortar slots ----
    double uvol[4];
    double asum = 0.0, thmin = 1.0;
    unsigned long long nf = 0, viol = 0;
    if (act) {
        double tf[4];
        tf[0] = a > 0 ? fmin(th, sTh[le][q - 1]) : 0.0;
        tf[1] = a < N ? fmin(th, sTh[le][q + 1]) : 0.0;
        tf[2] = b > 0 ? fmin(th, sTh[le][q - n]) : 0.0;
        tf[3] = b < N ? fmin(th, sTh[le][q + n]) : 0.0;
#pragma unroll
        for (int v = 0; v < 4; ++v)
            uvol[v] = uFV[v] + tf[0] * cf[0][v] + tf[1] * cf[1][v] + tf[2] * cf[2][v] + tf[3] * cf[3][v];
        if (a < N) {
            asum += 1.0 - tf[1];
            thmin = fmin(thmin, tf[1]);
            ++nf;
        }
        if (b < N) {
            asum += 1.0 - tf[3];
            thmin = fmin(thmin, tf[3]);
            ++nf;
        }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const size_t idx = ((size_t)e * 4 + v) * NN + q;
        double r = A.b * uvol[v];
        if (A.a != 0.0) r += A.a * A.un[idx];
        A.uout[idx] = r;
    }
    if (nmf == 0) {
        if (A.limiter != DGIDP_LIMIT_NONE && (uvol[0] < rmin || pressure(uvol, g) < pmin || uvol[0] != uvol[0]))
            viol = 1;
    } else {
        const double rt = rmin * kMargin, pt = pmin * kMargin;
        for (int j = 0; j < nmf; ++j) {
            double c[4], dc[4];
            bool fin = true;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                c[v] = dtm * dS[j][v];
                dc[v] = nmf * c[v];
                fin = fin && isfinite(dc[v]);
            }
            double ts = 1.0;
            if (A.limiter != DGIDP_LIMIT_NONE) {
                // the high-order mortar flux is undefined when the interpolated
                // state leaves the admissible set: the mortar keeps the low-order flux
                if (!fin) {
                    ts = 0.0;
                } else {
                    if (dc[0] < 0.0) ts = fmin(ts, fmax((rt - uvol[0]) / dc[0], 0.0));
                    ts = fmin(ts, theta_p(uvol, dc, pt, g));
                }
            }
            double* S = A.slot + (size_t)slotid[j] * kSlotW;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                S[v] = uvol[v];
                S[4 + v] = c[v];
            }
            S[8] = ts;
            S[9] = rmin;
            S[10] = pmin;
        }
    }
    }
    if (A.st) push_stats(A.st, inad, viol, thmin, asum, nf, false);
}

// ---------------------------------------------------------------------------
// mortar kernel: one thread per slot
// ---------------------------------------------------------------------------
template <int N>
__global__ __launch_bounds__(256) void k_mortar(const double* __restrict__ slot,
                                                const int* __restrict__ snode,
                                                const int* __restrict__ spart, int M,
                                                double* uout, double bcoef, double gamma,
                                                int limiter, DevStats* st)
{
    constexpr int n = N + 1, NN = n * n, NS = 3 * n;
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    unsigned long long viol = 0, nm = 0;
    double asum = 0.0, thmin = 1.0;
    if (s < M * NS) {
        const int S = s / NS;
        double t = 1.0;
        for (int j = 0; j < NS; ++j) t = fmin(t, slot[((size_t)S * NS + j) * kSlotW + 8]);
        if (s == S * NS) {
            asum = 1.0 - t;
            thmin = t;
            nm = 1;
        }
        const double* R = slot + (size_t)s * kSlotW;
        const int part = spart[s];
        bool apply = true;
        double corr[4] = {0, 0, 0, 0};
        if (t != 0.0)
#pragma unroll
            for (int v = 0; v < 4; ++v) corr[v] = t * R[4 + v];
        if (part >= 0) {
            const int S2 = part / NS;
            if (S2 < S) {
                apply = false;  // the lower-numbered mortar applies both corrections
            } else {
                double t2 = 1.0;
                for (int j = 0; j < NS; ++j) t2 = fmin(t2, slot[((size_t)S2 * NS + j) * kSlotW + 8]);
                if (t2 != 0.0)
#pragma unroll
                    for (int v = 0; v < 4; ++v) corr[v] += t2 * slot[(size_t)part * kSlotW + 4 + v];
            }
        }
        if (apply) {
            const int node = snode[s];
            const int e = node / NN, q = node - e * NN;
            double w[4];
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                uout[((size_t)e * 4 + v) * NN + q] += bcoef * corr[v];
                w[v] = R[v] + corr[v];
            }
            if (limiter != DGIDP_LIMIT_NONE &&
                (w[0] < R[9] || pressure(w, gamma) < R[10] || w[0] != w[0]))
                viol = 1;
        }
    }
    if (st) push_stats(st, 0, viol, thmin, asum, nm, true);
}

// ---------------------------------------------------------------------------
// time step: per node sum_j 2 d_ij / m_i (or the low-order estimate), grid max
// ---------------------------------------------------------------------------
struct DtArgs {
    const double* u;
    const int* fnbr;
    const int* fmort;
    const int* mort;
    const double* h;
    int E;
    double gamma, cfl;
    int mode;
    double* partial;
    unsigned int* counter;
    double* dt_out;
    DevStats* st;
};

template <int N>
__device__ __forceinline__ double wave_speed(const NodeP& s, int d)
{
    return fabs(d == 0 ? s.v1 : s.v2) + s.c;
}

template <int N>
__global__ __launch_bounds__(256) void k_dt(DtArgs A)
{
    constexpr int n = N + 1, NN = n * n, EPB = 256 / NN, NT = EPB * NN;
    __shared__ double sL[EPB][2][NN];
    __shared__ double sRed[4];
    __shared__ bool sLast;
    const Tab<N>& tb = T<N>();
    const double g = A.gamma;
    const int tid = threadIdx.x;
    const int le = tid / NN, q = tid - le * NN, a = q % n, b = q / n;
    const int e = blockIdx.x * EPB + le;
    const bool act = tid < NT && e < A.E;
    NodeP me;
    double hx = 1.0, hy = 1.0;
    if (act) {
        load_node<N>(A.u, e, q, me, g);
        hx = A.h[2 * e];
        hy = A.h[2 * e + 1];
        sL[le][0][q] = wave_speed<N>(me, 0);
        sL[le][1][q] = wave_speed<N>(me, 1);
    }
    __syncthreads();
    double s = 0.0;
    if (act) {
        if (A.mode == DGIDP_DT_LOWORDER) {
            s = (N + 1) * (sL[le][0][q] / hx + sL[le][1][q] / hy);
        } else {
            const double lx = sL[le][0][q], ly = sL[le][1][q];
            double sum = 0.0;
            if (a > 0) sum += 2.0 * tb.w[b] * hy * 0.25 * fmax(lx, sL[le][0][q - 1]);
            if (a < N) sum += 2.0 * tb.w[b] * hy * 0.25 * fmax(lx, sL[le][0][q + 1]);
            if (b > 0) sum += 2.0 * tb.w[a] * hx * 0.25 * fmax(ly, sL[le][1][q - n]);
            if (b < N) sum += 2.0 * tb.w[a] * hx * 0.25 * fmax(ly, sL[le][1][q + n]);
            const int kpos[4] = {b, b, a, a};
            const bool onf[4] = {a == 0, a == N, b == 0, b == N};
            for (int f = 0; f < 4; ++f) {
                if (!onf[f]) continue;
                const int k = kpos[f], d = f >> 1, code = A.fmort[e * 4 + f];
                const double hf = f < 2 ? hy : hx, lm = d == 0 ? lx : ly;
                if (code < 0) {
                    NodeP o;
                    load_node<N>(A.u, A.fnbr[e * 4 + f], face_q<N>(f ^ 1, k), o, g);
                    sum += 2.0 * tb.w[k] * hf * 0.25 * fmax(lm, wave_speed<N>(o, d));
                } else if (!fm_small(code)) {
                    const int S = fm_mortar(code);
                    for (int hh = 0; hh < 2; ++hh) {
                        const int sm = A.mort[S * 4 + 2 + hh];
                        for (int l = 0; l < n; ++l) {
                            const double wt = tb.Wt[k][hh * n + l];
                            if (wt == 0.0) continue;
                            NodeP o;
                            load_node<N>(A.u, sm, face_q<N>(f ^ 1, l), o, g);
                            sum += 2.0 * wt * hf * 0.25 * fmax(lm, wave_speed<N>(o, d));
                        }
                    }
                } else {
                    const int hh = fm_half(code), L = A.fnbr[e * 4 + f];
                    for (int j = 0; j < n; ++j) {
                        const double wt = tb.Wt[j][hh * n + k];
                        if (wt == 0.0) continue;
                        NodeP o;
                        load_node<N>(A.u, L, face_q<N>(f ^ 1, j), o, g);
                        sum += 2.0 * wt * (2.0 * hf) * 0.25 * fmax(lm, wave_speed<N>(o, d));
                    }
                }
            }
            s = sum / (0.25 * hx * hy * tb.w[a] * tb.w[b]);
        }
    }
    s = wave_max(s);
    if ((tid & 63) == 0) sRed[tid >> 6] = s;
    __syncthreads();
    if (tid == 0) {
        double m = fmax(fmax(sRed[0], sRed[1]), fmax(sRed[2], sRed[3]));
        A.partial[blockIdx.x] = m;
        __threadfence();
        const unsigned int done = atomicAdd(A.counter, 1u);
        sLast = (done == gridDim.x - 1);
    }
    __syncthreads();
    if (sLast) {
        // last block: reduce the per-block maxima, publish dt, re-arm the counter
        __threadfence();
        double m = 0.0;
        for (int i = tid; i < (int)gridDim.x; i += 256) m = fmax(m, __builtin_nontemporal_load(&A.partial[i]));
        m = wave_max(m);
        if ((tid & 63) == 0) sRed[tid >> 6] = m;
        __syncthreads();
        if (tid == 0) {
            m = fmax(fmax(sRed[0], sRed[1]), fmax(sRed[2], sRed[3]));
            const double dt = A.cfl / m;
            *A.dt_out = dt;
            if (A.st) A.st->dt = dt;
            *A.counter = 0u;
        }
    }
}

// ---------------------------------------------------------------------------
// small utility kernels
// ---------------------------------------------------------------------------
__global__ void k_permute(int E, int NN, const int* perm, const double* src, double* dst, int to_int)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t per = 4 * (size_t)NN;
    if (i >= (size_t)E * per) return;
    const int e = (int)(i / per);
    const size_t r = i - (size_t)e * per;
    const size_t j = (size_t)perm[e] * per + r;
    if (to_int) dst[i] = src[j];
    else dst[j] = src[i];
}

__global__ void k_set_double(double* p, double v) { *p = v; }

int launch_set_double(double* p, double v, hipStream_t s)
{
    hipLaunchKernelGGL(k_set_double, dim3(1), dim3(1), 0, s, p, v);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

__global__ void k_stats_reset(DevStats* st)
{
    st->fv_inadmissible = 0;
    st->violations = 0;
    st->theta_vol_min_bits = __double_as_longlong(1.0);
    st->theta_mort_min_bits = __double_as_longlong(1.0);
    st->alpha_vol_sum = 0.0;
    st->alpha_mort_sum = 0.0;
    st->nfaces = 0;
    st->nmortars = 0;
}

__global__ void k_check_state(int total_nodes, int NN, double g, const double* u, unsigned long long* bad)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= total_nodes) return;
    const int e = i / NN, q = i - e * NN;
    double w[4];
    for (int v = 0; v < 4; ++v) w[v] = u[((size_t)e * 4 + v) * NN + q];
    const double p = pressure(w, g);
    const bool ok = isfinite(w[0]) && isfinite(w[1]) && isfinite(w[2]) && isfinite(w[3]) &&
                    w[0] > 0.0 && p > 0.0;
    if (!ok) atomicMin(bad, (unsigned long long)i);
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
template <int N>
static int stage_N(const DevMesh& m, const KernelParams& kp, const double* uin, const double* un,
                   double* uout, double a, double b, const double* dt, DevStats* st, int mode,
                   hipStream_t s)
{
    constexpr int NN = (N + 1) * (N + 1), EPB = 256 / NN;
    StageArgs A;
    A.uin = uin;
    A.un = un;
    A.uout = uout;
    A.a = a;
    A.b = b;
    A.dt = dt;
    A.fnbr = m.fnbr;
    A.fmort = m.fmort;
    A.mort = m.mort;
    A.h = m.h;
    A.slot = m.slot;
    A.E = m.E;
    A.gamma = kp.gamma;
    A.beta = kp.beta;
    A.limiter = kp.limiter;
    A.st = st;
    const int grid = (m.E + EPB - 1) / EPB;
    const bool mixed = kp.precision == DGIDP_MIXED;
    if (mode == MODE_STAGE) {
        if (mixed) hipLaunchKernelGGL((k_stage<N, MODE_STAGE, true>), dim3(grid), dim3(256), 0, s, A);
        else hipLaunchKernelGGL((k_stage<N, MODE_STAGE, false>), dim3(grid), dim3(256), 0, s, A);
    } else if (mode == MODE_RHS_HIGH) {
        if (mixed) hipLaunchKernelGGL((k_stage<N, MODE_RHS_HIGH, true>), dim3(grid), dim3(256), 0, s, A);
        else hipLaunchKernelGGL((k_stage<N, MODE_RHS_HIGH, false>), dim3(grid), dim3(256), 0, s, A);
    } else {
        hipLaunchKernelGGL((k_stage<N, MODE_RHS_LOW, false>), dim3(grid), dim3(256), 0, s, A);
    }
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_stage(int N, const DevMesh& m, const KernelParams& kp, const double* uin,
                 const double* un, double* uout, double a, double b, const double* dt,
                 DevStats* st, hipStream_t s)
{
    if (m.E == 0) return 0;
    if (N == 3) return stage_N<3>(m, kp, uin, un, uout, a, b, dt, st, MODE_STAGE, s);
    if (N == 4) return stage_N<4>(m, kp, uin, un, uout, a, b, dt, st, MODE_STAGE, s);
    return -1;
}

int launch_rhs(int N, const DevMesh& m, const KernelParams& kp, const double* u, int which,
               double* du, hipStream_t s)
{
    if (m.E == 0) return 0;
    const int mode = which == DGIDP_RHS_HIGH ? MODE_RHS_HIGH : MODE_RHS_LOW;
    if (N == 3) return stage_N<3>(m, kp, u, nullptr, du, 0.0, 1.0, nullptr, nullptr, mode, s);
    if (N == 4) return stage_N<4>(m, kp, u, nullptr, du, 0.0, 1.0, nullptr, nullptr, mode, s);
    return -1;
}

int launch_mortar(int N, const DevMesh& m, double* uout, double b, DevStats* st, hipStream_t s,
                  double gamma, int limiter)
{
    if (m.M == 0) return 0;
    const int NS = 3 * (N + 1);
    const int total = m.M * NS;
    const int grid = (total + 255) / 256;
    if (N == 3)
        hipLaunchKernelGGL(k_mortar<3>, dim3(grid), dim3(256), 0, s, m.slot, m.slot_node,
                           m.slot_partner, m.M, uout, b, gamma, limiter, st);
    else if (N == 4)
        hipLaunchKernelGGL(k_mortar<4>, dim3(grid), dim3(256), 0, s, m.slot, m.slot_node,
                           m.slot_partner, m.M, uout, b, gamma, limiter, st);
    else
        return -1;
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int dt_blocks(int N, int E)
{
    const int EPB = 256 / ((N + 1) * (N + 1));
    return (E + EPB - 1) / EPB;
}

int launch_dt(int N, const DevMesh& m, const KernelParams& kp, const double* u, double cfl,
              int mode, double* partial, unsigned int* counter, int nblocks, double* dt_out,
              DevStats* st, hipStream_t s)
{
    DtArgs A;
    A.u = u;
    A.fnbr = m.fnbr;
    A.fmort = m.fmort;
    A.mort = m.mort;
    A.h = m.h;
    A.E = m.E;
    A.gamma = kp.gamma;
    A.cfl = cfl;
    A.mode = mode;
    A.partial = partial;
    A.counter = counter;
    A.dt_out = dt_out;
    A.st = st;
    if (N == 3) hipLaunchKernelGGL(k_dt<3>, dim3(nblocks), dim3(256), 0, s, A);
    else if (N == 4) hipLaunchKernelGGL(k_dt<4>, dim3(nblocks), dim3(256), 0, s, A);
    else return -1;
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_permute(int N, int E, const int* perm, const double* src, double* dst, int to_internal,
                   hipStream_t s)
{
    const int NN = (N + 1) * (N + 1);
    const size_t total = (size_t)E * 4 * NN;
    const int grid = (int)((total + 255) / 256);
    hipLaunchKernelGGL(k_permute, dim3(grid), dim3(256), 0, s, E, NN, perm, src, dst, to_internal);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_stats_reset(DevStats* st, hipStream_t s)
{
    hipLaunchKernelGGL(k_stats_reset, dim3(1), dim3(1), 0, s, st);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_check_state(int N, int E, double gamma, const double* u, unsigned long long* bad,
                       hipStream_t s)
{
    const int NN = (N + 1) * (N + 1);
    const int total = E * NN;
    hipLaunchKernelGGL(k_check_state, dim3((total + 255) / 256), dim3(256), 0, s, total, NN, gamma,
                       u, bad);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace dgidp
