// HIP kernels of dgidp for gfx950 (MI355X).
//
// One SSP-RK3 stage (Sec. 2.3 and Sec. 3 intro of the paper) is two kernels:
//   k_stage   one thread per LGL node; a block holds 4 elements in one wave
//             (N = 3) or 5 elements in two waves (N = 4).  It stages the element in LDS,
//             evaluates the surface fluxes with one lane per face node
//             (conforming LLF, Kopriva's L2 mortar, the sparse IDP mortar flux
//             of eq. interfaceflux_local), the Ranocha two-point fluxes once per
//             node pair of every line, telescopes them into high-order subcell
//             fluxes (eq. fluxdifferencingform), evaluates the LLF subcell
//             fluxes (eq. FVmethod), forms the low-order update and the
//             positivity bounds (eq. Bounds_Positivity), limits the volume
//             antidiffusive fluxes per subcell face and writes a u^n + b u^vol.
//             Nodes on mortars also leave a slot record with their mortar
//             antidiffusive increment and their own admissible fraction of it.
//   k_mortar  one thread per mortar slot: the mortar's factor is the minimum
//             over its slots (one factor per mortar keeps the flux conservative,
//             Sec. 2.3); corrections are added in ascending mortar order.
// The time step (eq. timestep_restriction) is a per-block max (k_dt) merged by
// one 64-bit atomic max per block into one of kDtSpread accumulators; the first
// stage kernel of the step reduces those and takes dt = cfl / max.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "dgidp_internal.h"
#include "dgidp_mlp_dev.h"

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
// the same ranges walked from their ends: a kernel that reads what the
// previous one wrote takes the most recently written batches, the ones most
// likely still held by the memory-side cache, first
__device__ __forceinline__ int xcd_batch_rev(int bid, int nb)
{
    const int q = nb >> 3, r = nb & 7;
    const int x = bid & 7, j = bid >> 3;
    const int len = x < r ? q + 1 : q;
    return (x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q) + len - 1 - j;
}

// launch geometry per degree: one-wave blocks of 4 elements at N = 3 (the
// phase barriers stay inside a wave and a late block holds less work),
// two-wave blocks of 5 elements at N = 4 (125 of 128 lanes busy; a block
// needs 19.6 KB of LDS, so eight blocks, sixteen waves, fill a compute unit
// to the four waves per SIMD that the conforming variant's registers allow).
// Three-wave blocks of 7 elements (175 of 192 lanes, 40 KB of LDS with all
// pairs stored at once, four blocks per CU) took 410.9 against 385.4 us per
// launch on the 246,736-leaf workload.
template <int N>
struct Geo {
    static constexpr int n = N + 1, NN = n * n;
    static constexpr int BS = N == 3 ? 64 : 128;   // block size
    static constexpr int EPB = BS / NN;            // 4 for N = 3, 5 for N = 4
    static_assert(EPB == stage_block_elems(N), "host element order assumes this block size");
    static constexpr int NT = EPB * NN;            // active threads
    static constexpr int NFN = 4 * n;              // face nodes per element
    static constexpr int NPL = n * (n - 1) / 2;    // node pairs per line
    static constexpr int NP = 2 * n * NPL;         // node pairs per element
    static constexpr int NF = 2 * N * n;           // interior subcell faces per element
    // LDS variable stride of the primitive array: unpadded.  At N = 3 padding
    // to an odd element stride cost blocks per compute unit, more than the
    // bank conflicts it saved; at N = 4 a pad of one made no difference
    // (288.7 against 289.8 us per stage on the 246,736-leaf workload).
    static constexpr int PR = NN;  // sR variable stride
    // x and y pairs in two passes where the x pairs fill whole thread rounds
    // (N = 4); the pair buffer then needs the larger of the mortar staging
    // (12 n) and half the pairs with the x lines' telescoped fluxes.  The
    // low-order subcell fluxes go to the primitive rows once those are read,
    // so the pair buffer no longer holds them.
    static constexpr bool SPLIT = (n * NPL) % NN == 0;
    static constexpr int XH = n * NPL;  // SPLIT: the x lines' telescoped fluxes follow the pair slots
    // (one pad slot at N = 4: an odd stride keeps the elements sharing a wave
    // out of step with the 256-byte bank period)
    static constexpr int PP = SPLIT ? (XH + n * N > 12 * n ? XH + n * N : 12 * n) + 1 : NP;  // sPair variable stride
    // free pair slots after the telescoping (the slots N..NPL-1 of every line
    // whose first N slots hold its telescoped fluxes) carry the surface terms
    // of the face nodes: face f, position k in line f L + k / FR, slot N + k % FR
    static constexpr int FR = NPL - N;
    static constexpr int FL = (n + FR - 1) / FR;
    static_assert(FR >= 1 && FL <= 2 && 4 * FL <= (SPLIT ? n : 2 * n), "surface-term slots");
    static __device__ __forceinline__ int fslot(int f, int k)
    {
        if constexpr (FL == 1) return f * NPL + N + k;
        else return (f * 2 + (k >= FR ? 1 : 0)) * NPL + N + (k >= FR ? k - FR : k);
    }
};

// (l, k) of the node pairs l < k of a line, 6 bits per pair in line order
template <int N>
constexpr unsigned long long pair_code()
{
    unsigned long long c = 0;
    int i = 0;
    for (int l = 0; l <= N; ++l)
        for (int k = l + 1; k <= N; ++k) {
            c |= (unsigned long long)(l | (k << 3)) << (6 * i);
            ++i;
        }
    return c;
}

// The node pairs of an element, N per thread: thread q evaluates the pairs
// q + i NN (i < N) of the list "x lines, then y lines; in each line the pairs
// (l, k), l < k, in order" (N NN pairs in all, 2 n n(n-1)/2).  Entry
// ql | qk << 5 | d << 10 | l << 11 | k << 14: the two nodes (element-local
// indices), the direction and their positions along the line.
template <int N>
struct PairMap {
    static constexpr int n = N + 1, NN = n * n, NPL = n * (n - 1) / 2;
    unsigned int code[NN][N];
    constexpr PairMap() : code()
    {
        for (int q = 0; q < NN; ++q)
            for (int i = 0; i < N; ++i) {
                const int p = q + i * NN;
                const int d = p / (n * NPL), rem = p % (n * NPL), line = rem / NPL;
                int l = 0, r = rem % NPL;
                while (r >= n - 1 - l) {
                    r -= n - 1 - l;
                    ++l;
                }
                const int k = l + 1 + r;
                const int ql = d == 0 ? line * n + l : l * n + line;
                const int qk = d == 0 ? line * n + k : k * n + line;
                code[q][i] = (unsigned)(ql | qk << 5 | d << 10 | l << 11 | k << 14);
            }
    }
};
__constant__ PairMap<3> c_pm3 = PairMap<3>();
__constant__ PairMap<4> c_pm4 = PairMap<4>();
template <int N>
__device__ __forceinline__ unsigned pair_entry(int q, int i);
template <>
__device__ __forceinline__ unsigned pair_entry<3>(int q, int i) { return c_pm3.code[q][i]; }
template <>
__device__ __forceinline__ unsigned pair_entry<4>(int q, int i) { return c_pm4.code[q][i]; }

// ---------------------------------------------------------------------------
// arithmetic helpers
// ---------------------------------------------------------------------------
// 1/y from the hardware estimate and two Newton steps (about 1 ulp); used on
// the paths every node takes, where y > 0
__device__ __forceinline__ double frcp(double y)
{
    double r = __builtin_amdgcn_rcp(y);
    double e = fma(-y, r, 1.0);
    r = fma(r, e, r);
    e = fma(-y, r, 1.0);
    return fma(r, e, r);
}

// sqrt(y) for y >= 0 (normal or zero): the hardware reciprocal square root,
// one step of the coupled Newton iteration for sqrt y and 1 / (2 sqrt y), then
// a Newton correction of the root (about 1 ulp).  y = 0 gives 0, y < 0 or NaN
// gives NaN.
__device__ __forceinline__ double fsqrt(double y)
{
    const double r = __builtin_amdgcn_rsq(y);
    double g = y * r, h = 0.5 * r;
    const double e = fma(-g, h, 0.5);
    g = fma(g, e, g);
    h = fma(h, e, h);
    g = fma(fma(-g, g, y), h, g);
    return y == 0.0 ? 0.0 : g;
}

// two FP32 values in one FP64 LDS slot (register moves only)
struct F2 {
    float x, y;
};
__device__ __forceinline__ double pack2(float x, float y)
{
    return __hiloint2double(__float_as_int(y), __float_as_int(x));
}
__device__ __forceinline__ F2 unpack2(double d)
{
    return F2{__int_as_float(__double2loint(d)), __int_as_float(__double2hiint(d))};
}

struct NodeP {
    double u[4];
    double r, v1, v2, p, c;
};

__device__ __forceinline__ void make_node(NodeP& s, double g)
{
    const double ir = frcp(s.u[0]);
    s.r = s.u[0];
    s.v1 = s.u[1] * ir;
    s.v2 = s.u[2] * ir;
    s.p = (g - 1.0) * (s.u[3] - 0.5 * (s.u[1] * s.v1 + s.u[2] * s.v2));
    s.c = fsqrt(g * s.p * ir);
}

// Ghost state across a boundary face f (0 x-, 1 x+, 2 y-, 3 y+) of the interior
// node s; the outward normal is the axis f / 2, negative on even faces.  Wall:
// the normal momentum reversed.  Characteristic, by the outward normal velocity
// vn and sound speed c of s: the exterior state x if vn <= -c; x's density and
// velocity with s's pressure if vn <= 0; s's density and velocity with x's
// pressure if vn < c; else s.  Outflow: s.
__device__ __forceinline__ void boundary_ghost(int kind, const double* x, const NodeP& s, int f,
                                               double g, double* gu)
{
    const int d = f >> 1;
#pragma unroll
    for (int v = 0; v < 4; ++v) gu[v] = s.u[v];
    if (kind == DGIDP_BC_WALL) {  // (constant indices keep gu in registers)
        if (d == 0) gu[1] = -s.u[1];
        else gu[2] = -s.u[2];
        return;
    }
    if (kind != DGIDP_BC_CHARACTERISTIC) return;
    const double vn = (f & 1) ? (d == 0 ? s.v1 : s.v2) : -(d == 0 ? s.v1 : s.v2);
    if (vn >= s.c) return;
    if (vn <= -s.c) {
#pragma unroll
        for (int v = 0; v < 4; ++v) gu[v] = x[v];
        return;
    }
    const double ixr = 1.0 / x[0], xv1 = x[1] * ixr, xv2 = x[2] * ixr;
    if (vn <= 0.0) {
        gu[0] = x[0];
        gu[1] = x[0] * xv1;
        gu[2] = x[0] * xv2;
        gu[3] = s.p / (g - 1.0) + 0.5 * x[0] * (xv1 * xv1 + xv2 * xv2);
    } else {
        const double xp = (g - 1.0) * (x[3] - 0.5 * (x[1] * xv1 + x[2] * xv2));
        gu[3] = xp / (g - 1.0) + 0.5 * s.r * (s.v1 * s.v1 + s.v2 * s.v2);
    }
}

__device__ __forceinline__ double pressure(const double* u, double g)
{
    return (g - 1.0) * (u[3] - 0.5 * (u[1] * u[1] + u[2] * u[2]) * frcp(u[0]));
}

// local Lax-Friedrichs flux across a face (eq. FVmethod): 1/2 (f_n(u_L) + f_n(u_R)) -
// 1/2 lambda (u_R - u_L), lambda = max(|v_n| + c) of the two states.
// Normal direction d and side are run-time values (lanes of a wave hold
// different faces): this element's state `own`, the other side's state `o`,
// own_low = this element is on the low side.  Branch free, so a wave evaluates
// one flux body whatever mix of faces its lanes hold.
__device__ __forceinline__ void llf_face(int d, bool own_low, const NodeP& own, const NodeP& o,
                                         double* F)
{
    const bool dx = d == 0;
    const double va = dx ? own.v1 : own.v2, vb = dx ? o.v1 : o.v2;
    const double lam = fmax(fabs(va) + own.c, fabs(vb) + o.c);
    const double hl = own_low ? 0.5 * lam : -0.5 * lam;
    double fa[4], fb[4];
    fa[0] = own.r * va;
    fa[1] = own.u[1] * va + (dx ? own.p : 0.0);
    fa[2] = own.u[2] * va + (dx ? 0.0 : own.p);
    fa[3] = (own.u[3] + own.p) * va;
    fb[0] = o.r * vb;
    fb[1] = o.u[1] * vb + (dx ? o.p : 0.0);
    fb[2] = o.u[2] * vb + (dx ? 0.0 : o.p);
    fb[3] = (o.u[3] + o.p) * vb;
#pragma unroll
    for (int v = 0; v < 4; ++v) F[v] = 0.5 * (fa[v] + fb[v]) - hl * (o.u[v] - own.u[v]);
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
    llf_face(d, large_low, ui, us, F);
}

// logarithmic mean x^ln = (x - y) / (ln x - ln y) from the logarithms lx, ly.
// Where |f| = |x - y| / (x + y) < 1e-2 (f^2 < 1e-4) the series
// x^ln = (x + y)/2 f / atanh f = (x + y)/2 (1 - f^2/3 - 4 f^4/45 - 44 f^6/945 - ...)
// (from the series of 2 atanh, as in Ismail & Roe 2009), whose next term is
// below 4e-18 relative there.  Branch free: one reciprocal serves whichever
// form applies.
__device__ __forceinline__ double lnmean(double x, double y, double lx, double ly)
{
    const double s = x + y, d = x - y;
    const bool ser = fabs(d) < 1e-2 * s;
    const double r = frcp(ser ? s : lx - ly);
    const double f = d * r, f2 = f * f;
    // 1/3 + f2 (4/45 + f2 44/945) = 44/945 (945/132 + f2 (21/11 + f2)): one
    // literal per instruction
    const double t = fma(f2, f2 + 21.0 / 11.0, 945.0 / 132.0) * f2;
    const double sv = 0.5 * s * fma(-44.0 / 945.0, t, 1.0);
    return ser ? sv : f;
}

// 1 / x^ln = (ln x - ln y) / (x - y); series (2 + f^2 (2/3 + f^2 (2/5 + f^2 2/7))) / (x + y)
__device__ __forceinline__ double inv_lnmean(double x, double y, double lx, double ly)
{
    const double s = x + y, d = x - y;
    const bool ser = fabs(d) < 1e-2 * s;
    const double r = frcp(ser ? s : d);
    const double f = d * r, f2 = f * f;
    // 2/3 + f2 (2/5 + f2 2/7) = 2/7 (7/3 + f2 (7/5 + f2))
    const double t = fma(f2, f2 + 7.0 / 5.0, 7.0 / 3.0) * f2;
    const double sv = fma(2.0 / 7.0, t, 2.0) * r;
    return ser ? sv : (lx - ly) * r;
}

// Natural logarithm for x > 0 normal (NaN for x <= 0 or NaN): x = m 2^k with
// m in [sqrt(1/2), sqrt(2)), f = m - 1 (exact), s = f / (2 + f), so that
// ln m = 2 atanh s = 2 s + T, T = 2 s^3/3 + 2 s^5/5 + ... (|s| < 0.172, the
// series to s^21 leaves less than 2^-56 of ln m), and 2 s = f - s f gives
// ln m = f - s (f - T / s) with T / s a polynomial in s^2; ln x = k ln 2 +
// ln m with ln 2 split into a head whose product with k is exact and a tail.
// About 1 ulp, thirty instructions (the run-time library's logarithm takes
// about eighty).
__device__ __forceinline__ double flog(double x)
{
    double m = __builtin_amdgcn_frexp_mant(x);  // [0.5, 1)
    int k = __builtin_amdgcn_frexp_exp(x);
    if (m < 0x1.6a09e667f3bcdp-1) {
        m *= 2.0;
        k -= 1;
    }
    const double f = m - 1.0;
    const double sf = f * frcp(2.0 + f);
    const double z = sf * sf;
    const double t = z * (2.0 / 3.0 + z * (2.0 / 5.0 + z * (2.0 / 7.0 + z * (2.0 / 9.0 + z * (2.0 / 11.0 +
                     z * (2.0 / 13.0 + z * (2.0 / 15.0 + z * (2.0 / 17.0 + z * (2.0 / 19.0 + z * (2.0 / 21.0))))))))));
    const double lm = f - sf * (f - t);
    const double kd = (double)k;
    const double r = fma(kd, 0x1.62e42fefp-1, fma(kd, 0x1.473de6af278edp-34, lm));
    return x > 0.0 ? r : __builtin_nan("");
}

__device__ __forceinline__ float lnmeanf(float x, float y, float lx, float ly)
{
    const float s = x + y, d = x - y;
    if (d * d < 1e-2f * (s * s)) {
        const float is = __builtin_amdgcn_rcpf(s);
        const float f2 = d * d * is * is;
        return s * __builtin_amdgcn_rcpf(2.0f + f2 * (2.0f / 3.0f + f2 * (2.0f / 5.0f + f2 * (2.0f / 7.0f))));
    }
    return d * __builtin_amdgcn_rcpf(lx - ly);
}

__device__ __forceinline__ float inv_lnmeanf(float x, float y, float lx, float ly)
{
    const float s = x + y, d = x - y;
    if (d * d < 1e-2f * (s * s)) {
        const float is = __builtin_amdgcn_rcpf(s);
        const float f2 = d * d * is * is;
        return (2.0f + f2 * (2.0f / 3.0f + f2 * (2.0f / 5.0f + f2 * (2.0f / 7.0f)))) * is;
    }
    return (lx - ly) * __builtin_amdgcn_rcpf(d);
}

// ---------------------------------------------------------------------------
// pressure blending factor: largest theta in [0,1] with rho(u0 + theta dc) > 0
// and p(u0 + theta dc) >= pt.  For rho > 0, p >= pt is
// g(theta) = (E - pt/(gamma-1)) rho - |m|^2 / 2 >= 0, a quadratic in theta whose
// admissible set along the ray is an interval [0, theta*] (p is concave).
// ---------------------------------------------------------------------------
// The ray's direction is S c (S = Gamma = 4 for the volume faces' increments,
// 1 otherwise): a power of two, so that S c is formed exactly inside the
// fused multiply-adds.
template <int S = 1>
__device__ __forceinline__ double theta_p(const double* u0, const double* c, double pt, double ig1)
{
    const double e0 = u0[3] - pt * ig1;
    const double g0 = u0[0] * e0 - 0.5 * (u0[1] * u0[1] + u0[2] * u0[2]);
    if (!(g0 > 0.0) || !(u0[0] > 0.0)) return 0.0;
    // full step admissible: the interval contains [0, 1]
    const double r1 = fma((double)S, c[0], u0[0]);
    if (r1 > 0.0) {
        const double m1 = fma((double)S, c[1], u0[1]), m2 = fma((double)S, c[2], u0[2]);
        const double g1v = fma((double)S, c[3], e0) * r1 - 0.5 * (m1 * m1 + m2 * m2);
        if (g1v >= 0.0) return 1.0;
    }
    const double dc[4] = {S * c[0], S * c[1], S * c[2], S * c[3]};
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
constexpr double kMarginHi = 1.0 - 0x1p-40;  // the same for upper bounds
// the mortar correction aims at half that margin: a node that the volume
// limiter left on its target keeps 2^-41 of room, instead of a zero or one
// mortar factor decided by the sign of a rounding error
constexpr double kMarginMortar = 1.0 + 0x1p-41;
constexpr double kMarginMortarHi = 1.0 - 0x1p-41;
// the local bounds hold for the low-order state only up to rounding (it is a
// convex combination of bar states in exact arithmetic): the bound check allows
// this relative slack for them
constexpr double kLocalTol = 1e-12;
// density increments (per node and step) this small relative to the density are
// not limited against the local density bounds
constexpr double kLocalNegl = 1e-14;

// ---------------------------------------------------------------------------
// local bounds (eq. Bounds_Barstates)
// ---------------------------------------------------------------------------
// Density and log specific entropy ln(p rho^-gamma) of the bar state of the
// low-order graph edge between this element's node `own` and the node `o`
// across a face of direction d (own_low: `own` on the low side).  The bar state
// (u_i + u_j)/2 - c_ij . (f_j - f_i) / (2 d_ij) with d_ij = |c_ij| lambda_ij is
// (u_L + u_R)/2 - (f(u_R) - f(u_L)) / (2 lambda), lambda as in llf_face.  A bar
// state outside the admissible set (only by rounding) gives -inf: no entropy
// bound from it.
__device__ __forceinline__ void bar_bounds(int d, bool own_low, const NodeP& own, const NodeP& o,
                                           double g, double& rb, double& lsb)
{
    const bool dx = d == 0;
    const double va = dx ? own.v1 : own.v2, vb = dx ? o.v1 : o.v2;
    const double lam = fmax(fabs(va) + own.c, fabs(vb) + o.c);
    const double k = (own_low ? 0.5 : -0.5) * frcp(lam);
    double fa[4], fb[4];
    fa[0] = own.r * va;
    fa[1] = own.u[1] * va + (dx ? own.p : 0.0);
    fa[2] = own.u[2] * va + (dx ? 0.0 : own.p);
    fa[3] = (own.u[3] + own.p) * va;
    fb[0] = o.r * vb;
    fb[1] = o.u[1] * vb + (dx ? o.p : 0.0);
    fb[2] = o.u[2] * vb + (dx ? 0.0 : o.p);
    fb[3] = (o.u[3] + o.p) * vb;
    double ub[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) ub[v] = 0.5 * (own.u[v] + o.u[v]) - k * (fb[v] - fa[v]);
    rb = ub[0];
    const double pb = (g - 1.0) * (ub[3] - 0.5 * (ub[1] * ub[1] + ub[2] * ub[2]) / ub[0]);
    lsb = (rb > 0.0 && pb > 0.0) ? log(pb) - g * log(rb) : -__builtin_inf();
}

// psi(theta) = p(u0 + theta dc) - exp(lst + gamma ln rho(theta)) and its
// derivative: psi >= 0 with rho > 0 is p rho^-gamma >= exp(lst).  p is concave
// in the conserved variables and rho^gamma convex, so psi is concave on the ray.
__device__ __forceinline__ double psi_s(const double* u0, const double* dc, double th, double lst,
                                        double g, double& dpsi)
{
    const double q0 = u0[0] + th * dc[0], q1 = u0[1] + th * dc[1];
    const double q2 = u0[2] + th * dc[2], q3 = u0[3] + th * dc[3];
    if (!(q0 > 0.0)) {
        dpsi = 0.0;
        return -__builtin_inf();
    }
    const double ir = 1.0 / q0;
    const double v1 = q1 * ir, v2 = q2 * ir;
    const double p = (g - 1.0) * (q3 - 0.5 * (q1 * v1 + q2 * v2));
    const double rg = exp(lst + g * log(q0));
    const double dp = (g - 1.0) * (dc[3] - v1 * dc[1] - v2 * dc[2] + 0.5 * (v1 * v1 + v2 * v2) * dc[0]);
    dpsi = dp - g * rg * ir * dc[0];
    return p - rg;
}

// Largest theta in [0, thi] with p rho^-gamma >= exp(lst) at u0 + theta dc, on
// a ray where rho stays positive up to thi.  The admissible set of the concave
// psi is an interval [0, theta*] when psi(0) >= 0.  The root is bracketed from
// both sides: the chord through the feasible and the infeasible end cuts the
// axis at or below theta* (concavity), the Newton step from the infeasible end
// at or above it (the tangent lies above psi); the two-sided iteration of
// convex limiting (Guermond, Nazarov, Popov and Tomas, SIAM J. Sci. Comput.
// 2018).  When the two estimates are within 1e-14 (or cross by rounding) it
// returns the chord point, theta* up to rounding; otherwise it stops when the
// bracket is that narrow, at most 16 rounds, and returns the feasible end;
// psi(0) <= 0 returns 0.
__device__ double theta_s(const double* u0, const double* dc, double lst, double g, double thi)
{
    if (!(thi > 0.0)) return 0.0;
    double dh, dl, dx;
    double ph = psi_s(u0, dc, thi, lst, g, dh);
    if (ph >= 0.0) return thi;
    double pl = psi_s(u0, dc, 0.0, lst, g, dl);
    if (!(pl > 0.0)) return 0.0;
    double lo = 0.0, hi = thi;
#pragma unroll 1
    for (int it = 0; it < 16; ++it) {
        double c = lo + pl * (hi - lo) / (pl - ph);
        double nw = dh < 0.0 ? hi - ph / dh : hi;
        if (!(c > lo)) c = lo;
        if (!(c < hi)) c = hi;
        if (!(nw < hi)) nw = hi;
        if (nw < c) nw = c;
        const double pc = psi_s(u0, dc, c, lst, g, dx);
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
        const double pn = psi_s(u0, dc, nw, lst, g, dx);
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

// Node factor of the volume limiter from the node's four face increments cf
// (dt/m_i-scaled, zero for missing faces): Zalesak factors for the density
// floor rfl (and, with local bounds, the ceiling rce), the pressure root per
// face and, with local bounds, the entropy root per face on [0, theta] (log
// entropy floor lsm); the last two on Gamma = 4-scaled increments.
template <bool LOCB>
__device__ __forceinline__ double volume_factor(const double* uFV, const double (&cf)[4][4], double rfl,
                                                double pfl, double rce, double lsm, double lsi, double g,
                                                double ig1)
{
    const double rt = rfl * kMargin, pt = pfl * kMargin;
    // Zalesak: the sum of the negative (positive) density increments may use at
    // most the distance to the floor (ceiling)
    double P = 0.0, Pp = 0.0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        P += fmin(cf[j][0], 0.0);
        if (LOCB) Pp += fmax(cf[j][0], 0.0);
    }
    // local bounds: increments below kLocalNegl of the density are rounding
    // noise and are not limited (a node whose density interval has zero width
    // would otherwise switch between theta = 0 and 1 on the sign of a rounding
    // error)
    if (LOCB && P > -kLocalNegl * uFV[0]) P = 0.0;
    if (LOCB && Pp < kLocalNegl * uFV[0]) Pp = 0.0;
    double th = 1.0;
    if (P < 0.0) th = fmax(fmin((rt - uFV[0]) * frcp(P), 1.0), 0.0);
    if (LOCB && Pp > 0.0) th = fmin(th, fmax((rce * kMarginHi - uFV[0]) / Pp, 0.0));
    // pressure: each face's increment scaled by Gamma = 2d = 4 (a zero
    // increment, as on a missing face, admits theta = 1 at an admissible uFV)
#pragma unroll
    for (int j = 0; j < 4; ++j) th = fmin(th, theta_p<4>(uFV, cf[j], pt, ig1));
    // specific entropy: per face on [0, th].  The target ln(s_min (1 + 2^-40))
    // is capped at lsi lowered by 2^-41: with bounds from the low-order solution
    // lsi is the node's own low-order log entropy (where the node itself is the
    // minimum of its neighbourhood, the raised bound would lie above the state
    // the limiter starts from); with bar states lsi = +inf (no cap)
    if (LOCB) {
        const double lst = fmin(lsm + 0x1p-40, lsi - 0x1p-41);
#pragma unroll 1
        for (int j = 0; j < 4; ++j) {
            const double dc[4] = {4.0 * cf[j][0], 4.0 * cf[j][1], 4.0 * cf[j][2], 4.0 * cf[j][3]};
            if (dc[0] == 0.0 && dc[1] == 0.0 && dc[2] == 0.0 && dc[3] == 0.0) continue;
            th = theta_s(uFV, dc, lst, g, th);
        }
    }
    return th;
}

// Factor of one mortar node for its n_i-scaled increment dc on top of u^vol:
// density floor (and ceiling), pressure root, entropy root, all against half
// the volume margin.
template <bool LOCB>
__device__ __forceinline__ double mortar_factor(const double* uvol, const double* dc, double rfl, double pfl,
                                                double rce, double lsm, double lsi, double g, double ig1)
{
    const double rt = rfl * kMarginMortar, pt = pfl * kMarginMortar;
    double ts = 1.0;
    const bool negl = LOCB && fabs(dc[0]) <= kLocalNegl * uvol[0];
    if (dc[0] < 0.0 && !negl) ts = fmin(ts, fmax((rt - uvol[0]) / dc[0], 0.0));
    if (LOCB && dc[0] > 0.0 && !negl) ts = fmin(ts, fmax((rce * kMarginMortarHi - uvol[0]) / dc[0], 0.0));
    ts = fmin(ts, theta_p(uvol, dc, pt, ig1));
    if (LOCB) ts = theta_s(uvol, dc, fmin(lsm + 0x1p-41, lsi - 0x1p-40), g, ts);
    return ts;
}

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

// accumulation of per-thread statistics, one atomic per wave; every lane of
// the wave must call it.  Counts are taken from lane masks (per lane: inad and
// viol 0 or 1, nf 0, 1 or 2); the two floating-point reductions run only in
// waves where some lane has a value to contribute.
__device__ __forceinline__ void push_stats(DevStats* st, unsigned long long inad,
                                           unsigned long long viol, double thmin, double asum,
                                           unsigned long long nf, bool mortar)
{
    const unsigned long long ninad = __popcll(__ballot(inad != 0));
    const unsigned long long nviol = __popcll(__ballot(viol != 0));
    const unsigned long long nfs = __popcll(__ballot(nf >= 1)) + __popcll(__ballot(nf >= 2));
    if (__ballot(asum != 0.0)) asum = wave_sum(asum);
    if (__ballot(thmin < 1.0)) thmin = wave_min(thmin);
    if ((threadIdx.x & 63) == 0) {
        if (ninad) atomicAdd(&st->fv_inadmissible, ninad);
        if (nviol) atomicAdd(&st->violations, nviol);
        if (nfs) {
            if (mortar) {
                atomicAdd(&st->alpha_mort_sum, asum);
                atomicAdd(&st->nmortars, nfs);
            } else {
                atomicAdd(&st->alpha_vol_sum, asum);
                atomicAdd(&st->nfaces, nfs);
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
    const double* ind;  // combined limiting: shock indicator per element, in [0, 1]
    const double* lob;  // bounds from the low-order solution: [E][3][NN] rho min, rho max, ln s min
    // when set, dt = cfl / max over the accumulator set dtmax (bits of
    // non-negative doubles); block 0 stores it in dt_out
    const unsigned long long* dtmax;
    double cfl;
    double* dt_out;
    const int* fnbr;
    const int* fnbr2;
    const int* fmort;
    const int* mort;
    const double* h;
    double* slot;
    const int8_t* bkind;  // boundary nodes: condition and exterior state
    const double* bext;
    // element batches of this launch: blist[boff + i], i < gridDim.x (the
    // batches holding a mortar element and the others are separate launches)
    const int* blist;
    int boff;
    int E;
    double gamma, beta;
    double ig1;  // 1 / (gamma - 1)
    int rev;     // walk the XCD batch ranges from their ends (conforming variant only)
    int limiter;
    int vflux;  // two-point volume flux: DGIDP_FLUX_RANOCHA or DGIDP_FLUX_CHANDRASHEKAR
    DevStats* st;
};

// node (a, b) at position k along face f
template <int N>
__device__ __forceinline__ int face_q(int f, int k)
{
    constexpr int n = N + 1;
    // x faces (0, 1) run along a column, y faces (2, 3) along a row; the odd
    // face of each pair is N columns or N rows further on
    const int hi = f & 1;
    return f < 2 ? k * n + hi * N : k + hi * (N * n);
}

template <int N>
__device__ __forceinline__ void load_u(const double* u, int e, int q, double* w)
{
    constexpr int NN = (N + 1) * (N + 1);
    // one address per node; the variables at constant offsets (index < 2^30, mesh limit)
    const double* p = u + ((unsigned)e * 4u * NN + (unsigned)q);
#pragma unroll
    for (int v = 0; v < 4; ++v) w[v] = p[v * NN];
}

template <int N>
__device__ __forceinline__ void load_node(const double* u, int e, int q, NodeP& s, double g)
{
    load_u<N>(u, e, q, s.u);
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

// node qq of the block's element le from its LDS primitives; the conserved
// state is formed again from them (rho v = rho * v, E = p / (gamma - 1) +
// (rho v . v) / 2: within a few ulp of the stored state, the same for every
// reader of a node, so that equal states still meet in a zero flux difference)
#define LDS_NODE(X, qq)                                                    \
    do {                                                                   \
        X.r = sR[le][0][qq];                                               \
        X.v1 = sR[le][1][qq];                                              \
        X.v2 = sR[le][2][qq];                                              \
        X.p = sR[le][3][qq];                                               \
        X.c = sR[le][4][qq];                                               \
        X.u[0] = X.r;                                                      \
        X.u[1] = X.r * X.v1;                                               \
        X.u[2] = X.r * X.v2;                                               \
        X.u[3] = fma(X.p, ig1, 0.5 * (X.u[1] * X.v1 + X.u[2] * X.v2));     \
    } while (0)

// LIMK: 0 positivity (or none, at run time), 1 local bounds from bar states,
// 2 the blend of positivity and bar-state local factors by the per-element
// shock indicator A.ind (eq. combination_posLim_local), 3 local bounds from the
// low-order solution (eq. Bounds_LowOrder), read from A.lob
// MORT: the launch over the element batches that hold a mortar element (the
// surface phase with Kopriva's mortar and the sparse low-order mortar flux,
// mortar slot records); the batches without one run the MORT = false variant,
// which has no mortar code, fewer registers and four waves per SIMD.
template <int N, int MODE, bool MIXED, int LIMK, bool MORT>
// at least three waves per SIMD: the local-limiting variant would otherwise
// take 172 registers and run two (63.3 against 67.7 us on the 22,156-leaf
// blast with a few spilled registers; the other variants fit anyway); the
// conforming positivity variant fits 128 registers, four waves
__global__ __launch_bounds__(Geo<N>::BS) __attribute__((amdgpu_waves_per_eu((!MORT && LIMK == 0) ? 4 : 3)))
void k_stage(StageArgs A)
{
    using G = Geo<N>;
    // LOC: local bounds enforced; COMB: blended with positivity; BAR: the bounds
    // come from bar states (computed here), otherwise from the low-order
    // solution (read from A.lob); PURE: local factors only
    constexpr bool LOC = LIMK >= 1, COMB = LIMK == 2, BAR = LIMK == 1 || LIMK == 2;
    constexpr bool PURE = LIMK == 1 || LIMK == 3;
    constexpr int n = G::n, NN = G::NN, EPB = G::EPB, NT = G::NT, NFN = G::NFN;
    constexpr int NPL = G::NPL, NP = G::NP, NF = G::NF, PPT = NP / NN, PP = G::PP;
    static_assert(NP % NN == 0, "pair split");
    constexpr bool DSTAT = (n * NPL) % NN == 0, SPLIT = G::SPLIT;
    constexpr int XH = n * NPL;  // SPLIT: the x lines' telescoped fluxes follow the pair slots
    static_assert(!SPLIT || (DSTAT && XH + n * N <= G::PP), "two-pass pair buffer");
    static_assert(G::PP >= 12 * n, "mortar buffers reuse the pair buffer");
    static_assert(G::PR == NN && 4 * NF + NN <= 8 * NN, "subcell fluxes and node factors reuse sR");
    constexpr int MB = 4 * n;  // offset of the mortar-node fluxes in the pair buffer

    // variable-major (see Geo)
    __shared__ double sR[EPB][8][G::PR];     // rho, v1, v2, p, c, ln rho, z = rho/p, ln z
    __shared__ double sPair[EPB][4][G::PP];  // pair fluxes, then telescoped fluxes and surface terms
    // bar states of local limiting: rows 0-3 the subcell faces owned by a node
    // (x: density, log entropy; y: the same), rows 4-6 the face lanes' range
    // across the element face; row 0 later the local node factors of the blend
    __shared__ double sB[BAR ? EPB : 1][7][BAR ? NN : 1];
    __shared__ double sTw[2][n];              // LGL weights and their reciprocals, read per lane
    __shared__ double sS[n][n];               // Sbar, read per pair
    // After phase 5b the primitive rows of sR are read no more: they take the
    // low-order subcell fluxes, variable-major over the NF faces (x faces
    // b N + a, y faces N n + a N + b), and after them the node factors.
#define sFV(v, fi) sRe[(v) * NF + (fi)]
#define sTh(qq) sRe[4 * NF + (qq)]

    const Tab<N>& tb = T<N>();
    const double g = A.gamma, ig1 = A.ig1;
    const int tid = threadIdx.x;
    const int le = tid / NN, q = tid - le * NN, a = q % n, b = q / n;
    const int xb = !MORT && A.rev ? xcd_batch_rev(blockIdx.x, gridDim.x) : xcd_batch(blockIdx.x, gridDim.x);
    const int e = (A.blist ? A.blist[A.boff + xb] : xb) * EPB + le;
    double* const sRe = &sR[0][0][0] + le * 8 * NN;  // element le's rows, flat
    double* const sPe = &sPair[0][0][0] + le * 4 * PP;  // element le's pair buffer, flat
    const bool act = tid < NT && e < A.E;
    if (tid < n) {
        sTw[0][tid] = tb.w[tid];
        sTw[1][tid] = tb.winv[tid];
    }
    if (tid < NN) (&sS[0][0])[tid] = (&tb.S[0][0])[tid];

    // ---- phase 1: own node into LDS; face-node role and its remote loads ----
    double hx = 1.0, hy = 1.0;
    int fcode[4] = {-1, -1, -1, -1};
    const bool fnode = act && q < NFN;       // this lane also evaluates one face node
    const int ff = q / n, fk = q - (q / n) * n;  // its face and position
    const int qfo = face_q<N>(ff, fk), qfn = face_q<N>(ff ^ 1, fk);  // the face node, its neighbour's
    int fcode_f = -1, fnb = 0, fnb2 = -1, bk = 0;
    double onb[4];  // conforming neighbour state (boundary: exterior state) across face ff at fk
    double us1[4];  // large side: the second small element's trace at position fk
    // u^n of this node for the SSP combination, loaded where it is needed (so
    // that it occupies no registers through the flux phases), and this node's
    // state (uin)
    double un4[4] = {0, 0, 0, 0};
    double u0[4] = {0, 0, 0, 0};
    // the low-order surface term of this lane's face node, kept in registers
    // until phase 5 frees pair slots, which then carry it to the node's own thread
    double fterm[4] = {0, 0, 0, 0};
    // local bounds: own log entropy; for face lanes the density range and the
    // smallest log entropy of the bar states across this lane's face node
    double ls_own = 0.0;
    double w_e = 0.0;  // combined limiting: weight of the local factors
    bool need_loc = false;  // this element computes bounds and local factors (uniform per element)
    double fb_lo = __builtin_inf(), fb_hi = -__builtin_inf(), fb_ls = __builtin_inf();
    const double dtpart =
        A.dtmax ? __longlong_as_double((long long)A.dtmax[(tid & 63) * kDtStride]) : 0.0;
    // this thread's node pairs (the pair map), loaded with the state
    unsigned pcode[PPT];
#pragma unroll
    for (int i = 0; i < PPT; ++i) pcode[i] = act ? pair_entry<N>(q, i) : 0u;
    if (act) {
        // issue the independent global loads first
#pragma unroll
        for (int f = 0; f < 4; ++f) fcode[f] = A.fmort[e * 4 + f];
        if (fnode) {
            fnb = A.fnbr[e * 4 + ff];
            fnb2 = A.fnbr2[e * 4 + ff];
        }
        NodeP me;
        load_node<N>(A.uin, e, q, me, g);
        hx = A.h[2 * e];
        hy = A.h[2 * e + 1];
        if (COMB) w_e = A.ind[e];
#pragma unroll
        for (int v = 0; v < 4; ++v) u0[v] = me.u[v];
        // the logarithms feed only the two-point volume fluxes: FP32 in the
        // mixed mode, where rows 5-7 hold the FP32 operands of those fluxes in
        // pairs (rho, p), (ln rho, z), (ln z, 0)
        const double z = me.r * frcp(me.p);
        sR[le][0][q] = me.r;
        sR[le][1][q] = me.v1;
        sR[le][2][q] = me.v2;
        sR[le][3][q] = me.p;
        sR[le][4][q] = me.c;
        double lr, lz;
        if (MIXED) {
            const float lrf = __logf((float)me.r), lzf = __logf((float)z);
            lr = lrf;
            lz = lzf;
            sR[le][5][q] = pack2((float)me.r, (float)me.p);
            sR[le][6][q] = pack2(lrf, (float)z);
            sR[le][7][q] = pack2(lzf, 0.0f);
        } else {
            lr = flog(me.r);
            lz = flog(z);
            sR[le][5][q] = lr;
            sR[le][6][q] = z;
            sR[le][7][q] = lz;
        }
        // the blend needs local factors only where the indicator fires, and at
        // mortar nodes (their mortar may blend with another element's weight)
        need_loc = LOC && (!COMB || w_e > 0.0 || fcode[0] >= 0 || fcode[1] >= 0 || fcode[2] >= 0 ||
                           fcode[3] >= 0);
        // ln(p rho^-gamma) of the node itself, the bar state (i, i)
        if (need_loc) ls_own = MIXED ? log(me.p) - g * log(me.r) : (1.0 - g) * lr - lz;
        if (fnode) {
            fcode_f = fcode[ff];
            if (fcode_f == -1) {
                load_u<N>(A.uin, fnb, qfn, onb);
            } else if (fcode_f < -1) {
                const int j = (-2 - fcode_f) * n + fk;
                bk = A.bkind[j];
#pragma unroll
                for (int v = 0; v < 4; ++v) onb[v] = A.bext[(size_t)j * 4 + v];
            } else if (MORT && !fm_small(fcode_f)) {
                // large side: both small traces at position fk, kept in
                // registers for the mortar-node fluxes and staged for the
                // sparse low-order pairs of the other positions
                load_u<N>(A.uin, fnb, qfn, onb);
                load_u<N>(A.uin, fnb2, qfn, us1);
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    sPair[le][v][MB + (ff * 2 + 0) * n + fk] = onb[v];
                    sPair[le][v][MB + (ff * 2 + 1) * n + fk] = us1[v];
                }
            } else if (MORT) {
                // small side: stage the large face trace for the interpolation
                double w[4];
                load_u<N>(A.uin, fnb, qfn, w);
#pragma unroll
                for (int v = 0; v < 4; ++v) sPair[le][v][ff * n + fk] = w[v];
            }
        }
    }
    __syncthreads();
    double dt;
    if (A.dtmax) {
        const double m = wave_max(dtpart);
        dt = A.cfl / m;
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            *A.dt_out = dt;
            if (A.st) A.st->dt = dt;
        }
    } else {
        dt = A.dt ? *A.dt : 0.0;
    }

    // ---- phase 2: one surface flux per face node ----
    const int dff = ff >> 1;
    const bool lowf = ff & 1;                    // element on the low side of face ff
    const double sgf = lowf ? -1.0 : 1.0;
    const double hff = ff < 2 ? hy : hx;
    if (fnode) {
        NodeP own;  // the face node's state
        LDS_NODE(own, qfo);
        if (fcode_f < 0) {
            NodeP o;
            if (fcode_f == -1) {
#pragma unroll
                for (int v = 0; v < 4; ++v) o.u[v] = onb[v];
            } else {
                boundary_ghost(bk, onb, own, ff, g, o.u);
            }
            make_node(o, g);
            double F[4];
            llf_face(dff, lowf, own, o, F);
            if (BAR && need_loc) {
                bar_bounds(dff, lowf, own, o, g, fb_lo, fb_ls);
                fb_hi = fb_lo;
            }
            const double W = sgf * sTw[0][fk] * hff * 0.5;
#pragma unroll
            for (int v = 0; v < 4; ++v) fterm[v] = W * F[v];
        } else if (MORT && !fm_small(fcode_f)) {
            // large side: mortar-node fluxes at position fk of both halves
            // (kept in registers until every lane has read the staged small
            // traces), and the sparse low-order pairs of this node
            for (int hh = 0; hh < 2; ++hh) {
                NodeP ui, us;
#pragma unroll
                for (int v = 0; v < 4; ++v) us.u[v] = hh == 0 ? onb[v] : us1[v];
                make_node(us, g);
                // the large face interpolated to half hh, from the face nodes'
                // conserved states formed as LDS_NODE does
                double ia[4] = {0, 0, 0, 0};
#pragma unroll
                for (int j = 0; j < n; ++j) {
                    const int qj = face_q<N>(ff, j);
                    const double r = sR[le][0][qj], v1 = sR[le][1][qj], v2 = sR[le][2][qj];
                    const double m1 = r * v1, m2 = r * v2;
                    const double uj[4] = {r, m1, m2, fma(sR[le][3][qj], ig1, 0.5 * (m1 * v1 + m2 * v2))};
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        if (MIXED) ia[v] = (float)ia[v] + tb.If[hh][fk][j] * (float)uj[v];
                        else ia[v] += tb.I[hh][fk][j] * uj[v];
                    }
                }
#pragma unroll
                for (int v = 0; v < 4; ++v) ui.u[v] = ia[v];
                make_node(ui, g);
                double F[4];
                mortar_flux(dff, lowf, ui, us, F);
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    if (hh == 0) onb[v] = F[v];
                    else us1[v] = F[v];
                }
            }
            // (over this node's nonzero weights only: a wave runs as many
            // rounds as its busiest lane)
            double lo[4] = {0, 0, 0, 0};
            const int nz = tb.lnc[fk];
#pragma unroll 1
            for (int i = 0; i < nz; ++i) {
                const int col = tb.lnz[fk][i];  // h n + l
                const double wt = tb.Wt[fk][col];
                NodeP us;
#pragma unroll
                for (int v = 0; v < 4; ++v) us.u[v] = sPair[le][v][MB + ff * 2 * n + col];
                make_node(us, g);
                double Gf[4];
                llf_face(dff, lowf, own, us, Gf);
                if (BAR && need_loc) {
                    double rb, lb;
                    bar_bounds(dff, lowf, own, us, g, rb, lb);
                    fb_lo = fmin(fb_lo, rb);
                    fb_hi = fmax(fb_hi, rb);
                    fb_ls = fmin(fb_ls, lb);
                }
                const double W = sgf * wt * hff * 0.5;
#pragma unroll
                for (int v = 0; v < 4; ++v) lo[v] += W * Gf[v];
            }
#pragma unroll
            for (int v = 0; v < 4; ++v) fterm[v] = lo[v];
        } else if (MORT) {
            // small side: interpolate the large face, LLF on the mortar = this face
            const int hh = fm_half(fcode_f);
            NodeP ui;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                if (MIXED) {
                    float acc = 0.0f;
#pragma unroll
                    for (int j = 0; j < n; ++j) acc += tb.If[hh][fk][j] * (float)sPair[le][v][ff * n + j];
                    ui.u[v] = acc;
                } else {
                    double acc = 0.0;
#pragma unroll
                    for (int j = 0; j < n; ++j) acc += tb.I[hh][fk][j] * sPair[le][v][ff * n + j];
                    ui.u[v] = acc;
                }
            }
            make_node(ui, g);
            double F[4], ho[4], lo[4] = {0, 0, 0, 0};
            mortar_flux(dff, !lowf, ui, own, F);
#pragma unroll
            for (int v = 0; v < 4; ++v) ho[v] = sgf * sTw[0][fk] * hff * 0.5 * F[v];
            const int nz = tb.snc[hh][fk];
#pragma unroll 1
            for (int i = 0; i < nz; ++i) {
                const int j = tb.snz[hh][fk][i];
                const double wt = tb.Wt[j][hh * n + fk];
                NodeP uj;
#pragma unroll
                for (int v = 0; v < 4; ++v) uj.u[v] = sPair[le][v][ff * n + j];
                make_node(uj, g);
                double Gf[4];
                llf_face(dff, lowf, own, uj, Gf);
                if (BAR && need_loc) {
                    double rb, lb;
                    bar_bounds(dff, lowf, own, uj, g, rb, lb);
                    fb_lo = fmin(fb_lo, rb);
                    fb_hi = fmax(fb_hi, rb);
                    fb_ls = fmin(fb_ls, lb);
                }
                const double W = sgf * wt * hff;  // wt * h_L / 2 with h_L = 2 h
#pragma unroll
                for (int v = 0; v < 4; ++v) lo[v] += W * Gf[v];
            }
#pragma unroll
            for (int v = 0; v < 4; ++v) fterm[v] = lo[v];
            {
                const int S = fm_mortar(fcode_f);
                double* R = A.slot + (size_t)(S * 3 * n + n + fm_half(fcode_f) * n + fk) * kSlotW;
#pragma unroll
                for (int v = 0; v < 4; ++v) R[4 + v] = ho[v] - lo[v];
            }
        }
    }
    if constexpr (MORT) {  // (every batch of the mortar launch holds a mortar element)
        __syncthreads();
        // ---- phase 3: large sides publish and project the mortar fluxes ----
        const bool large = fnode && fcode_f >= 0 && !fm_small(fcode_f);
        if (large) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                sPair[le][v][MB + (ff * 2 + 0) * n + fk] = onb[v];
                sPair[le][v][MB + (ff * 2 + 1) * n + fk] = us1[v];
            }
        }
        __syncthreads();
        if (large) {
            const int S = fm_mortar(fcode_f);
            double ho[4];
#pragma unroll 1
            for (int v = 0; v < 4; ++v) {
                double acc = 0.0;
                if (MIXED) {
                    float accf = 0.0f;
#pragma unroll
                    for (int hh = 0; hh < 2; ++hh)
#pragma unroll
                        for (int l = 0; l < n; ++l)
                            accf += tb.Pf[hh][fk][l] * (float)sPair[le][v][MB + (ff * 2 + hh) * n + l];
                    acc = accf;
                } else {
#pragma unroll
                    for (int hh = 0; hh < 2; ++hh)
#pragma unroll
                        for (int l = 0; l < n; ++l)
                            acc += tb.P[hh][fk][l] * sPair[le][v][MB + (ff * 2 + hh) * n + l];
                }
                ho[v] = sgf * sTw[0][fk] * hff * 0.5 * acc;
            }
            double* R = A.slot + (size_t)(S * 3 * n + fk) * kSlotW;
#pragma unroll
            for (int v = 0; v < 4; ++v) R[4 + v] = ho[v] - fterm[v];
        }
        __syncthreads();
    }

    // ---- phase 4: two-point volume fluxes, once per node pair of each line ----
    // Each flux is evaluated in the frame of its pair's direction d: the normal
    // velocity is read from LDS row 1 + d and the tangential one from row 2 - d,
    // and the two momentum components are stored back to rows 1 + d and 2 - d,
    // so that lanes holding x and y pairs run the same instructions.
    // pair p = q + i NN: the x pairs are slots below n NPL.  Where NN divides that
    // count (N = 4) the direction of round i is a constant, and the x and y pairs
    // are evaluated in two passes (SPLIT): the x lines are telescoped into the
    // slots after the x pairs, then the y pairs take the x pairs' slots, so the
    // pair buffer holds half the pairs at a time.
    const double hhx = 0.5 * hy, hhy = 0.5 * hx;  // pair scale of x and y lines
    auto pair_rounds = [&](auto i0c, auto i1c, int slot_off) {
        constexpr int i0 = decltype(i0c)::value, i1 = decltype(i1c)::value;
        if (!act) return;
#pragma unroll
        for (int i = i0; i < i1; ++i) {
            const unsigned c = pcode[i];
            const int ql = c & 31, qk = (c >> 5) & 31;
            // a round wholly below or above the x pairs' n NPL slots has a constant
            // direction; only a round that straddles them (N = 3: the second) decodes it
            const int d = (i + 1) * NN <= n * NPL ? 0 : (i * NN >= n * NPL ? 1 : (int)((c >> 10) & 1));
            const int p = q + i * NN - slot_off;
            const int rn = 1 + d, rt = 2 - d;
            const double scale = sS[(c >> 11) & 7][(c >> 14) & 7] * (d ? hhy : hhx);
            const double Ln = sR[le][rn][ql], Lt = sR[le][rt][ql];
            const double Rn = sR[le][rn][qk], Rt = sR[le][rt][qk];
            double f0, fn, ft, f3;
            if (!MIXED) {
                const double L0 = sR[le][0][ql], L3 = sR[le][3][ql];
                const double L5 = sR[le][5][ql], L6 = sR[le][6][ql], L7 = sR[le][7][ql];
                const double R0 = sR[le][0][qk], R3 = sR[le][3][qk];
                const double R5 = sR[le][5][qk], R6 = sR[le][6][qk], R7 = sR[le][7][qk];
                const double iz_ln = inv_lnmean(L6, R6, L7, R7);
                const double vna = 0.5 * (Ln + Rn), vta = 0.5 * (Lt + Rt);
                const double fr = lnmean(L0, R0, L5, R5) * vna;
                f0 = fr;
                if (A.vflux == DGIDP_FLUX_CHANDRASHEKAR) {
                    // Chandrashekar: beta = z / 2, so p~ = rho-bar / (2 beta-bar) =
                    // (rho_L + rho_R) / (z_L + z_R) and 1 / (2 beta^ln) = 1 / z^ln
                    const double pt = (L0 + R0) * frcp(L6 + R6);
                    fn = fr * vna + pt;
                    ft = fr * vta;
                    f3 = fr * (ig1 * iz_ln - 0.25 * (Ln * Ln + Lt * Lt + Rn * Rn + Rt * Rt)) + vna * fn + vta * ft;
                } else {
                    fn = fr * vna + 0.5 * (L3 + R3);
                    ft = fr * vta;
                    f3 = fr * (0.5 * (Ln * Rn + Lt * Rt) + ig1 * iz_ln) + 0.5 * (L3 * Rn + R3 * Ln);
                }
            } else {
                const F2 L5 = unpack2(sR[le][5][ql]), L6 = unpack2(sR[le][6][ql]);
                const F2 R5 = unpack2(sR[le][5][qk]), R6 = unpack2(sR[le][6][qk]);
                const float L7 = unpack2(sR[le][7][ql]).x, R7 = unpack2(sR[le][7][qk]).x;
                const float rL = L5.x, rR = R5.x, pL = L5.y, pR = R5.y, zL = L6.y, zR = R6.y;
                const float iz_ln = inv_lnmeanf(zL, zR, L7, R7);
                const float vnL = (float)Ln, vnR = (float)Rn, vtL = (float)Lt, vtR = (float)Rt;
                const float vna = 0.5f * (vnL + vnR), vta = 0.5f * (vtL + vtR);
                const float fr = lnmeanf(rL, rR, L6.x, R6.x) * vna;
                f0 = fr;
                if (A.vflux == DGIDP_FLUX_CHANDRASHEKAR) {
                    const float pt = (rL + rR) / (zL + zR);
                    const float fnf = fr * vna + pt, ftf = fr * vta;
                    fn = fnf;
                    ft = ftf;
                    f3 = fr * ((float)ig1 * iz_ln - 0.25f * (vnL * vnL + vtL * vtL + vnR * vnR + vtR * vtR)) +
                         vna * fnf + vta * ftf;
                } else {
                    fn = fr * vna + 0.5f * (pL + pR);
                    ft = fr * vta;
                    f3 = fr * (0.5f * (vnL * vnR + vtL * vtR) + (float)ig1 * iz_ln) + 0.5f * (pL * vnR + pR * vnL);
                }
            }
            sPair[le][0][p] = scale * f0;
            sPair[le][rn][p] = scale * fn;
            sPair[le][rt][p] = scale * ft;
            sPair[le][3][p] = scale * f3;
        }
    };
    // telescoped high-order subcell fluxes of one line and variable: the flux
    // through the subcell face after position pos is the sum of the line's pair
    // fluxes (l, k) with l <= pos < k; with the position a loop constant every
    // pair index is static.  P: the line's pair slots; the N sums go to H.
    auto telescope = [&](const double* P, double* H) {
        double hof[N];
#pragma unroll
        for (int pos = 0; pos < N; ++pos) {
            double acc = 0.0;
#pragma unroll
            for (int l = 0; l <= pos; ++l)
#pragma unroll
                for (int k = pos + 1; k < n; ++k) acc += P[l * (2 * n - l - 1) / 2 + (k - l - 1)];
            hof[pos] = acc;
        }
#pragma unroll
        for (int pos = 0; pos < N; ++pos) H[pos] = hof[pos];
    };
    if constexpr (SPLIT) {
        // ---- phase 4 and 5a in two passes: one task per line and variable ----
        pair_rounds(std::integral_constant<int, 0>(), std::integral_constant<int, PPT / 2>(), 0);
        __syncthreads();
        if (act && q < 4 * n) telescope(&sPair[le][q & 3][(q >> 2) * NPL], &sPair[le][q & 3][XH + (q >> 2) * N]);
        __syncthreads();
        pair_rounds(std::integral_constant<int, PPT / 2>(), std::integral_constant<int, PPT>(), n * NPL);
        __syncthreads();
        if (act && q < 4 * n) {
            double* P = &sPair[le][q & 3][(q >> 2) * NPL];
            telescope(P, P);
        }
    } else {
        pair_rounds(std::integral_constant<int, 0>(), std::integral_constant<int, PPT>(), 0);
        __syncthreads();

        // ---- phase 5a: telescoped high-order subcell fluxes ----
        // One task per line and variable (x lines first, then y lines; 8n tasks,
        // task t = q + j NN for j = 0, 1).  The N sums replace the line's first N
        // pair slots of that variable, which no other task reads.
        static_assert(8 * n <= 2 * NN, "two telescoping tasks per lane at most");
        if (act) {
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                const int t = q + j * NN;
                if (t < 8 * n) {
                    double* P = &sPair[le][t & 3][(t >> 2) * NPL];
                    telescope(P, P);
                }
            }
        }
    }
    // ---- phase 5b: low-order subcell fluxes of the faces owned by this node,
    // x (a|a+1) and y (b|b+1) ----
    double FVo[2][4];
    double brb[2] = {0.0, 0.0}, bls[2] = {0.0, 0.0};  // bar state of each owned subcell face
    if (act) {
        NodeP me;
        LDS_NODE(me, q);
#pragma unroll
        for (int d = 0; d < 2; ++d) {
            const int pos = d == 0 ? a : b;
            if (pos >= N) continue;
            const int qn = d == 0 ? q + 1 : q + n;
            NodeP o;
            LDS_NODE(o, qn);
            double F[4];
            llf_face(d, true, me, o, F);
            if (BAR && need_loc) bar_bounds(d, true, me, o, g, brb[d], bls[d]);
            const double hs = 0.5 * (d == 0 ? hy : hx);
#pragma unroll
            for (int v = 0; v < 4; ++v) FVo[d][v] = hs * F[v];
        }
    }
    // every read of the primitives (and of the pairs, by the telescoping) is done
    __syncthreads();
    if (act) {
        if (a < N) {
#pragma unroll
            for (int v = 0; v < 4; ++v) sFV(v, b * N + a) = FVo[0][v];
        }
        if (b < N) {
#pragma unroll
            for (int v = 0; v < 4; ++v) sFV(v, N * n + a * N + b) = FVo[1][v];
        }
    }
    // the face lanes' surface terms go to the free pair slots
    if (fnode) {
        const int fs = G::fslot(ff, fk);
#pragma unroll
        for (int v = 0; v < 4; ++v) sPair[le][v][fs] = fterm[v];
    }
    if (BAR && need_loc) {
        if (a < N) {
            sB[le][0][q] = brb[0];
            sB[le][1][q] = bls[0];
        }
        if (b < N) {
            sB[le][2][q] = brb[1];
            sB[le][3][q] = bls[1];
        }
        if (fnode) {
            sB[le][4][q] = fb_lo;
            sB[le][5][q] = fb_hi;
            sB[le][6][q] = fb_ls;
        }
    }
    __syncthreads();

    // ---- phase 6: low-order residual, bounds, node factors ----
    if (act && MODE == MODE_STAGE && A.a != 0.0) load_u<N>(A.un, e, q, un4);
    const bool onf[4] = {a == 0, a == N, b == 0, b == N};
    // the four subcell faces j of the node (left, right, below, above), each
    // taken at a clamped in-range position of the node's own line; a missing
    // face (on the element boundary) has weight 0.  Face index (x faces
    // b N + pos, y faces N n + a N + pos), slot of the telescoped high-order
    // flux (x faces on line b, y faces on line a) and signed weight (+w on the
    // left / lower face, -w on the right / upper one), formed where used.
    auto fpos = [&](int j) {
        return j == 0 ? (a > 0 ? a - 1 : 0) : j == 1 ? (a < N ? a : N - 1) : j == 2 ? (b > 0 ? b - 1 : 0)
                                                                             : (b < N ? b : N - 1);
    };
    auto fidx = [&](int j) { return j < 2 ? b * N + fpos(j) : N * n + a * N + fpos(j); };
    auto hslot = [&](int j) {
        if (SPLIT) return j < 2 ? XH + b * N + fpos(j) : a * NPL + fpos(j);
        return j < 2 ? b * NPL + fpos(j) : (n + a) * NPL + fpos(j);
    };
    auto fweight = [&](int j) {
        const double w = sTw[0][j < 2 ? b : a];
        const bool has = j == 0 ? a > 0 : j == 1 ? a < N : j == 2 ? b > 0 : b < N;
        return has ? ((j & 1) ? -w : w) : 0.0;
    };
    double RLO[4], dS0[4] = {0, 0, 0, 0}, dS1[4] = {0, 0, 0, 0};
    int slot0 = -1, slot1 = -1, nmf = 0;
    double im = 1.0;  // 1 / m_i
    // antidiffusive flux w (f^HO - f^FV) of face j, signed as its weight, variable v
    auto antidiff = [&](int j, int v) { return fweight(j) * (sPe[v * PP + hslot(j)] - sFV(v, fidx(j))); };
    if (act) {
        im = 4.0 * frcp(hx * hy) * sTw[1][a] * sTw[1][b];
        const double cw[4] = {fweight(0), fweight(1), fweight(2), fweight(3)};
        const int fi[4] = {fidx(0), fidx(1), fidx(2), fidx(3)};
        // the surface terms of the element faces the node lies on: at most one
        // x face (0 or 1) and one y face (2 or 3), weight 0 where it lies on none
        const double csx = onf[0] || onf[1] ? 1.0 : 0.0, csy = onf[2] || onf[3] ? 1.0 : 0.0;
        const int fsx = G::fslot(a == 0 ? 0 : 1, b), fsy = G::fslot(b == 0 ? 2 : 3, a);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            double r = 0.0;
#pragma unroll
            for (int j = 0; j < 4; ++j) r = fma(cw[j], sFV(v, fi[j]), r);
            r = fma(csx, sPe[v * PP + fsx], r);
            r = fma(csy, sPe[v * PP + fsy], r);
            RLO[v] = r;
        }
        if constexpr (MORT) {
            // a node lies on at most one x face (a = 0 or N) and one y face (b = 0 or
            // N): slot 0 takes the mortar of its x face, slot 1 that of its y face
            const int cx = onf[0] ? fcode[0] : (onf[1] ? fcode[1] : -1);
            const int cy = onf[2] ? fcode[2] : (onf[3] ? fcode[3] : -1);
            auto slot_of = [&](int code, int k) {
                const int S3 = fm_mortar(code) * 3 * n;
                return fm_small(code) ? S3 + n + fm_half(code) * n + k : S3 + k;
            };
            if (cx >= 0) {
                slot0 = slot_of(cx, b);
#pragma unroll
                for (int v = 0; v < 4; ++v) dS0[v] = A.slot[(size_t)slot0 * kSlotW + 4 + v];
            }
            if (cy >= 0) {
                slot1 = slot_of(cy, a);
#pragma unroll
                for (int v = 0; v < 4; ++v) dS1[v] = A.slot[(size_t)slot1 * kSlotW + 4 + v];
            }
            nmf = (cx >= 0) + (cy >= 0);
        }
    }
    if (MODE == MODE_RHS_LOW || MODE == MODE_RHS_HIGH) {
        if (act) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                double r = RLO[v];
                if (MODE == MODE_RHS_HIGH) {
                    r += antidiff(0, v) + antidiff(1, v) + antidiff(2, v) + antidiff(3, v);
                    r += dS0[v] + dS1[v];
                }
                A.uout[((unsigned)e * 4u + v) * NN + q] = r * im;
            }
        }
        return;
    }

    const double dtm = dt * im;
    double uFV[4], cf[4][4];
    double rmin = 0.0, pmin = 0.0, th = 1.0;
    // local bounds: density floor (the larger of the local and the positivity
    // floor), ceiling, log entropy floor; thl the local node factor of the blend
    double rlf = 0.0, rhi = 0.0, lsm = 0.0, thl = 1.0;
    double lsi = 0.0;  // local bounds: the node's own low-order log entropy (cap of the entropy target)
    unsigned long long inad = 0;
    if (act) {
#pragma unroll
        for (int v = 0; v < 4; ++v) uFV[v] = u0[v] + dtm * RLO[v];
        const double pFV = pressure(uFV, g);
        if (!(uFV[0] > 0.0) || !(pFV > 0.0)) inad = 1;
        rmin = A.beta * uFV[0];
        pmin = A.beta * pFV;
        if (need_loc && !BAR) {
            // bounds from the low-order solution; the node's own low-order
            // state, as computed here, is inside them by definition (the
            // bounds kernel's copy of it may differ in the last bit)
            const size_t bi = (size_t)e * 3 * NN + q;
            double rlo = fmin(A.lob[bi], uFV[0]);
            rhi = fmax(A.lob[bi + NN], uFV[0]);
            lsm = A.lob[bi + 2 * NN];
            lsi = uFV[0] > 0.0 && pFV > 0.0 ? log(pFV) - g * log(uFV[0]) : -__builtin_inf();
            lsm = fmin(lsm, lsi);
            rlf = fmax(rmin, rlo);
        } else if (need_loc) {
            // bounds over the node and the bar states of its low-order neighbours
            // (the node's own bar state is its input state: no cap)
            lsi = __builtin_inf();
            double rlo = u0[0];
            rhi = u0[0];
            lsm = ls_own;
            if (a > 0) {
                rlo = fmin(rlo, sB[le][0][q - 1]);
                rhi = fmax(rhi, sB[le][0][q - 1]);
                lsm = fmin(lsm, sB[le][1][q - 1]);
            }
            if (a < N) {
                rlo = fmin(rlo, sB[le][0][q]);
                rhi = fmax(rhi, sB[le][0][q]);
                lsm = fmin(lsm, sB[le][1][q]);
            }
            if (b > 0) {
                rlo = fmin(rlo, sB[le][2][q - n]);
                rhi = fmax(rhi, sB[le][2][q - n]);
                lsm = fmin(lsm, sB[le][3][q - n]);
            }
            if (b < N) {
                rlo = fmin(rlo, sB[le][2][q]);
                rhi = fmax(rhi, sB[le][2][q]);
                lsm = fmin(lsm, sB[le][3][q]);
            }
            const int fnq[4] = {0 * n + b, 1 * n + b, 2 * n + a, 3 * n + a};  // face lane of each face
#pragma unroll
            for (int f = 0; f < 4; ++f) {
                if (!onf[f]) continue;
                rlo = fmin(rlo, sB[le][4][fnq[f]]);
                rhi = fmax(rhi, sB[le][5][fnq[f]]);
                lsm = fmin(lsm, sB[le][6][fnq[f]]);
            }
            // the positivity floor stays: the density floor is the larger one
            rlf = fmax(rmin, rlo);
        }
        // the faces' increments dt / m_i w (f^HO - f^FV), signed (zero for missing faces)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const double wd = dtm * fweight(j);
#pragma unroll
            for (int v = 0; v < 4; ++v) cf[j][v] = wd * (sPe[v * PP + hslot(j)] - sFV(v, fidx(j)));
        }
        if (A.limiter != DGIDP_LIMIT_NONE) {
            if (PURE) {
                th = volume_factor<true>(uFV, cf, rlf, pmin, rhi, lsm, lsi, g, ig1);
            } else {
                th = volume_factor<false>(uFV, cf, rmin, pmin, 0.0, 0.0, 0.0, g, ig1);
                if (COMB && need_loc) thl = volume_factor<true>(uFV, cf, rlf, pmin, rhi, lsm, lsi, g, ig1);
            }
        }
    }
    // the blend keeps its local node factors in the first bar-state row, read
    // above for the bounds
    if (COMB) __syncthreads();
    if (act) {
        sTh(q) = th;
        if (COMB) sB[le][0][q] = thl;
    }
    __syncthreads();

    // ---- phase 7: limited volume update, SSP combination, mortar slots ----
    double asum = 0.0, thmin = 1.0;
    unsigned long long nf = 0, viol = 0;
    if (act) {
        double uvol[4];
        double tf[4];
        // face factor: the smaller of its two node factors; blended:
        // (1 - w) theta_pos + w theta_local
        // (a missing face reads the node itself; its increment is zero)
        const int qn4[4] = {a > 0 ? q - 1 : q, a < N ? q + 1 : q, b > 0 ? q - n : q, b < N ? q + n : q};
#pragma unroll
        for (int j = 0; j < 4; ++j)
            tf[j] = COMB ? (1.0 - w_e) * fmin(th, sTh(qn4[j])) + w_e * fmin(thl, sB[le][0][qn4[j]])
                         : fmin(th, sTh(qn4[j]));
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
        double* po = A.uout + ((unsigned)e * 4u * NN + (unsigned)q);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            // (un4 is zero where a = 0: the first stage's input is u^n itself)
            po[v * NN] = fma(A.a, un4[v], A.b * uvol[v]);
        }
        if (nmf == 0) {
            if (PURE) {
                if (A.st && (!(uvol[0] >= rlf * (1.0 - kLocalTol)) || uvol[0] > rhi * (1.0 + kLocalTol) ||
                             pressure(uvol, g) < pmin ||
                             !(log(pressure(uvol, g)) - g * log(uvol[0]) >= lsm - kLocalTol)))
                    viol = 1;
            } else if (A.limiter != DGIDP_LIMIT_NONE) {
                // p(uvol) >= pmin as 2 rho (E - pmin / (gamma - 1)) >= |m|^2 (rho >= rmin > 0)
                const double gp = 2.0 * uvol[0] * (uvol[3] - pmin * ig1) - (uvol[1] * uvol[1] + uvol[2] * uvol[2]);
                if (!(uvol[0] >= rmin) || !(gp >= 0.0)) viol = 1;
            }
        } else {
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                if ((j == 0 ? slot0 : slot1) < 0) continue;
                const double* dS = j == 0 ? dS0 : dS1;
                double c[4], dc[4];
                bool fin = true;
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    c[v] = dtm * dS[v];
                    dc[v] = nmf * c[v];
                    fin = fin && isfinite(dc[v]);
                }
                double ts = 1.0, tsl = 1.0;
                if (A.limiter != DGIDP_LIMIT_NONE) {
                    // an undefined high-order mortar flux keeps the low-order flux
                    if (!fin) {
                        ts = tsl = 0.0;
                    } else if (PURE) {
                        ts = mortar_factor<true>(uvol, dc, rlf, pmin, rhi, lsm, lsi, g, ig1);
                    } else {
                        ts = mortar_factor<false>(uvol, dc, rmin, pmin, 0.0, 0.0, 0.0, g, ig1);
                        if (COMB) tsl = mortar_factor<true>(uvol, dc, rlf, pmin, rhi, lsm, lsi, g, ig1);
                    }
                }
                double* S = A.slot + (size_t)(j == 0 ? slot0 : slot1) * kSlotW;
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    S[v] = uvol[v];
                    S[4 + v] = c[v];
                }
                S[8] = ts;
                S[9] = PURE ? rlf : rmin;
                S[10] = pmin;
                if (PURE) {
                    S[11] = rhi;
                    S[12] = lsm;
                }
                if (COMB) {
                    S[13] = tsl;
                    S[14] = w_e;
                }
            }
        }
    }
    if (A.st) push_stats(A.st, inad, viol, thmin, asum, nf, false);
}

// ---------------------------------------------------------------------------
// mortar kernel: one thread per slot
// ---------------------------------------------------------------------------
// factor of mortar S: the minimum of its slots' node factors; combined
// limiting blends the positivity and the local minimum with the largest
// indicator of the mortar's three elements
template <int N>
__device__ __forceinline__ double mortar_theta(const double* __restrict__ slot, int S, int limiter)
{
    constexpr int NS = 3 * (N + 1);
    double t = 1.0, tl = 1.0, w = 0.0;
#pragma unroll
    for (int j = 0; j < NS; ++j) {
        const double* R = slot + ((size_t)S * NS + j) * kSlotW;
        t = fmin(t, R[8]);
        if (limiter == DGIDP_LIMIT_COMBINED) {
            tl = fmin(tl, R[13]);
            w = fmax(w, R[14]);
        }
    }
    return limiter == DGIDP_LIMIT_COMBINED ? (1.0 - w) * t + w * tl : t;
}

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
        // every load that needs no other load first: slot factors of the
        // mortar, this slot's record, its node and its partner
        const double* R = slot + (size_t)s * kSlotW;
        const int part = spart[s];
        const int node = snode[s];
        double rec[11];
#pragma unroll
        for (int i = 0; i < 11; ++i) rec[i] = R[i];
        double t = mortar_theta<N>(slot, S, limiter);
        const int e = node / NN, q = node - e * NN;
        double uo[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) uo[v] = uout[((size_t)e * 4 + v) * NN + q];
        if (s == S * NS) {
            asum = 1.0 - t;
            thmin = t;
            nm = 1;
        }
        bool apply = true;
        double corr[4] = {0, 0, 0, 0};
        if (t != 0.0)
#pragma unroll
            for (int v = 0; v < 4; ++v) corr[v] = t * rec[4 + v];
        if (part >= 0) {
            const int S2 = part / NS;
            if (S2 < S) {
                apply = false;  // the lower-numbered mortar applies both corrections
            } else {
                const double t2 = mortar_theta<N>(slot, S2, limiter);
                if (t2 != 0.0)
#pragma unroll
                    for (int v = 0; v < 4; ++v) corr[v] += t2 * slot[(size_t)part * kSlotW + 4 + v];
            }
        }
        if (apply) {
            double w[4];
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                uout[((size_t)e * 4 + v) * NN + q] = uo[v] + bcoef * corr[v];
                w[v] = rec[v] + corr[v];
            }
            if (limiter == DGIDP_LIMIT_LOCAL || limiter == DGIDP_LIMIT_LOCAL_LOWORDER) {
                const double rhi = R[11], lsm = R[12];
                const double pw = pressure(w, gamma);
                if (!(w[0] >= rec[9] * (1.0 - kLocalTol)) || w[0] > rhi * (1.0 + kLocalTol) ||
                    pw < rec[10] || !(log(pw) - gamma * log(w[0]) >= lsm - kLocalTol))
                    viol = 1;
            } else if (limiter != DGIDP_LIMIT_NONE &&
                       (w[0] < rec[9] || pressure(w, gamma) < rec[10] || w[0] != w[0])) {
                viol = 1;
            }
        }
    }
    if (st) push_stats(st, 0, viol, thmin, asum, nm, true);
}

// ---------------------------------------------------------------------------
// local bounds from the low-order solution (eq. Bounds_LowOrder): per node the
// density range over u^FV = u + dt R_LO / m of the node and its low-order
// neighbours (subcell neighbours; the matching node across a conforming face;
// the nodes with a nonzero sparse weight across a mortar; none across a
// boundary), and the smallest ln(p rho^-gamma) among those with rho, p > 0.
// Two passes: k_lowsol forms each node's low-order density and log entropy
// once (two logarithms per node, coalesced), k_lowbounds gathers them.
// ---------------------------------------------------------------------------
struct LoBoundsArgs {
    const double* u;
    const double* dlo;  // R_LO / m, [E][4][NN] (internal order)
    const double* dt;   // dt source as for the stage kernel: dt, or cfl / max(dtmax)
    const unsigned long long* dtmax;
    double cfl;
    const int* fnbr;
    const int* fnbr2;
    const int* fmort;
    int E;
    double gamma;
    double* lsv;  // [E][2][NN] low-order density, ln s (+inf where rho or p <= 0)
    double* lob;  // [E][3][NN] rho min, rho max, ln s min
};

template <int N>
__global__ __launch_bounds__(256) void k_lowsol(LoBoundsArgs A)
{
    constexpr int NN = (N + 1) * (N + 1);
    double dt;
    if (A.dtmax) {  // the same value the stage kernel derives (every lane takes part)
        const double part = __longlong_as_double((long long)A.dtmax[(threadIdx.x & 63) * kDtStride]);
        dt = A.cfl / wave_max(part);
    } else {
        dt = *A.dt;
    }
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (size_t)A.E * NN) return;
    const size_t e = i / NN, q = i - e * NN;
    double w[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const size_t k = (e * 4 + v) * NN + q;
        w[v] = A.u[k] + dt * A.dlo[k];
    }
    const double p = pressure(w, A.gamma);
    A.lsv[e * 2 * NN + q] = w[0];
    A.lsv[e * 2 * NN + NN + q] =
        w[0] > 0.0 && p > 0.0 ? log(p) - A.gamma * log(w[0]) : __builtin_inf();
}

template <int N>
__device__ __forceinline__ void lo_gather(const double* __restrict__ lsv, int e, int q, double& lo,
                                          double& hi, double& ls)
{
    constexpr int NN = (N + 1) * (N + 1);
    const double r = lsv[(size_t)e * 2 * NN + q];
    lo = fmin(lo, r);
    hi = fmax(hi, r);
    ls = fmin(ls, lsv[(size_t)e * 2 * NN + NN + q]);
}

// one thread per node
template <int N>
__global__ __launch_bounds__(256) void k_lowbounds(LoBoundsArgs A)
{
    constexpr int n = N + 1, NN = n * n;
    const Tab<N>& tb = T<N>();
    // (contiguous node ranges per XCD: the neighbours' values mostly in the same L2)
    const size_t i = (size_t)xcd_batch(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (i >= (size_t)A.E * NN) return;
    const int e = (int)(i / NN), q = (int)(i - (size_t)e * NN), a = q % n, b = q / n;
    double lo = __builtin_inf(), hi = -__builtin_inf(), ls = __builtin_inf();
    lo_gather<N>(A.lsv, e, q, lo, hi, ls);
    if (a > 0) lo_gather<N>(A.lsv, e, q - 1, lo, hi, ls);
    if (a < N) lo_gather<N>(A.lsv, e, q + 1, lo, hi, ls);
    if (b > 0) lo_gather<N>(A.lsv, e, q - n, lo, hi, ls);
    if (b < N) lo_gather<N>(A.lsv, e, q + n, lo, hi, ls);
    const bool on[4] = {a == 0, a == N, b == 0, b == N};
#pragma unroll
    for (int f = 0; f < 4; ++f) {
        if (!on[f]) continue;
        const int code = A.fmort[e * 4 + f];
        if (code < -1) continue;  // boundary
        const int k = f < 2 ? b : a;
        const int nb = A.fnbr[e * 4 + f];
        if (code == -1) {
            lo_gather<N>(A.lsv, nb, face_q<N>(f ^ 1, k), lo, hi, ls);
        } else if (!fm_small(code)) {
            const int nb2 = A.fnbr2[e * 4 + f];
#pragma unroll
            for (int hh = 0; hh < 2; ++hh)
#pragma unroll
                for (int l = 0; l < n; ++l)
                    if (tb.Wt[k][hh * n + l] != 0.0)
                        lo_gather<N>(A.lsv, hh == 0 ? nb : nb2, face_q<N>(f ^ 1, l), lo, hi, ls);
        } else {
            const int hh = fm_half(code);
#pragma unroll
            for (int kk = 0; kk < n; ++kk)
                if (tb.Wt[kk][hh * n + k] != 0.0) lo_gather<N>(A.lsv, nb, face_q<N>(f ^ 1, kk), lo, hi, ls);
        }
    }
    const size_t bi = (size_t)e * 3 * NN + q;
    A.lob[bi] = lo;
    A.lob[bi + NN] = hi;
    A.lob[bi + 2 * NN] = ls;
}

int launch_lowbounds(int N, const DevMesh& m, double gamma, const double* u, const double* dlo,
                     const DtSource& dt, double* lsv, double* lob, hipStream_t s)
{
    if (m.E == 0) return 0;
    LoBoundsArgs A;
    A.u = u;
    A.dlo = dlo;
    A.dt = dt.dt;
    A.dtmax = dt.dtmax;
    A.cfl = dt.cfl;
    A.fnbr = m.fnbr;
    A.fnbr2 = m.fnbr2;
    A.fmort = m.fmort;
    A.E = m.E;
    A.gamma = gamma;
    A.lsv = lsv;
    A.lob = lob;
    const size_t nodes = (size_t)m.E * (N + 1) * (N + 1);
    const dim3 grid((unsigned)((nodes + 255) / 256));
    if (N == 3) {
        hipLaunchKernelGGL(k_lowsol<3>, grid, dim3(256), 0, s, A);
        hipLaunchKernelGGL(k_lowbounds<3>, grid, dim3(256), 0, s, A);
    } else if (N == 4) {
        hipLaunchKernelGGL(k_lowsol<4>, grid, dim3(256), 0, s, A);
        hipLaunchKernelGGL(k_lowbounds<4>, grid, dim3(256), 0, s, A);
    } else {
        return -1;
    }
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

// ---------------------------------------------------------------------------
// time step: per node sum_j 2 d_ij / m_i (or the low-order estimate), block max
// ---------------------------------------------------------------------------
struct DtArgs {
    const double* u;
    const int* fnbr;
    const int* fnbr2;
    const int* fmort;
    const int* mort;
    const double* h;
    const int8_t* bkind;
    const double* bext;
    int E;
    double gamma;
    int mode;
    unsigned long long* acc;    // running maximum, bits of a non-negative double
    unsigned long long* other;  // the other accumulator, cleared for the next step
};

__device__ __forceinline__ double wave_speed(const NodeP& s, int d)
{
    return fabs(d == 0 ? s.v1 : s.v2) + s.c;
}

// the dt kernel: kDtBlock = 256-thread blocks (16 elements at N = 3, 10 at N = 4), fewer
// blocks and so fewer atomics than the stage kernel's geometry
// threads per block of the dt kernel (whole elements per block)
constexpr int kDtBlock = 256;

template <int N>
struct DtGeo {
    static constexpr int n = N + 1, NN = n * n, NFN = 4 * n;
    static constexpr int BS = kDtBlock, EPB = BS / NN, NT = EPB * NN;
};

template <int N>
__global__ __launch_bounds__(kDtBlock) void k_dt(DtArgs A)
{
    using G = DtGeo<N>;
    constexpr int n = G::n, NN = G::NN, EPB = G::EPB, NT = G::NT, NFN = G::NFN;
    __shared__ double sL[EPB][2][NN];
    __shared__ double sF[EPB][NFN];
    __shared__ double sMl[EPB][8 * n];  // wave speeds across mortars, staged per position
    constexpr int NW = G::BS / 64;  // waves per block
    __shared__ double sRed[NW];
    __shared__ double sTw[2][n];  // LGL weights and their reciprocals, read per lane
    const Tab<N>& tb = T<N>();
    const double g = A.gamma;
    const int tid = threadIdx.x;
    const int le = tid / NN, q = tid - le * NN, a = q % n, b = q / n;
    // (contiguous element ranges per XCD, as in the stage kernel: the face
    // neighbours' traces are then mostly in the same L2; each range from its
    // end, where the stage before this kernel finished writing)
    const int e = xcd_batch_rev(blockIdx.x, gridDim.x) * EPB + le;
    const bool act = tid < NT && e < A.E;
    if (tid < n) {
        sTw[0][tid] = tb.w[tid];
        sTw[1][tid] = tb.winv[tid];
    }
    const bool idp = A.mode != DGIDP_DT_LOWORDER;
    const bool fnode = act && idp && q < NFN;
    const int ff = q / n, fk = q - (q / n) * n, dff = ff >> 1;
    double hx = 1.0, hy = 1.0, lo_nb = 0.0;
    int code = -1, nb = 0, nb2 = -1;
    if (act) {
        if (fnode) {  // face tables first: the neighbour loads depend on them
            code = A.fmort[e * 4 + ff];
            nb = A.fnbr[e * 4 + ff];
            nb2 = A.fnbr2[e * 4 + ff];
        }
        NodeP me;
        load_node<N>(A.u, e, q, me, g);
        hx = A.h[2 * e];
        hy = A.h[2 * e + 1];
        sL[le][0][q] = wave_speed(me, 0);
        sL[le][1][q] = wave_speed(me, 1);
        if (fnode) {
            NodeP o;
            if (code >= -1) {
                load_node<N>(A.u, nb, face_q<N>(ff ^ 1, fk), o, g);
            } else {  // boundary: the ghost state of the face node
                const int j = (-2 - code) * n + fk;
                double x[4];
#pragma unroll
                for (int v = 0; v < 4; ++v) x[v] = A.bext[(size_t)j * 4 + v];
                NodeP s;
                load_node<N>(A.u, e, face_q<N>(ff, fk), s, g);
                boundary_ghost(A.bkind[j], x, s, ff, g, o.u);
                make_node(o, g);
            }
            lo_nb = wave_speed(o, dff);
            if (code >= 0) {
                // mortar: stage the wave speeds of the other side at position fk
                // (large side: both small elements; small side: the large one)
                sMl[le][(ff * 2) * n + fk] = lo_nb;
                if (!fm_small(code)) {
                    NodeP o2;
                    load_node<N>(A.u, nb2, face_q<N>(ff ^ 1, fk), o2, g);
                    sMl[le][(ff * 2 + 1) * n + fk] = wave_speed(o2, dff);
                }
            }
        }
    }
    __syncthreads();
    if (fnode) {
        // edges across face ff at position fk: 2 |c_ij| lambda_ij
        const double hf = ff < 2 ? hy : hx;
        const double lm = sL[le][dff][face_q<N>(ff, fk)];
        double sum = 0.0;
        if (code < 0) {
            sum = 0.5 * sTw[0][fk] * hf * fmax(lm, lo_nb);
        } else if (!fm_small(code)) {
#pragma unroll
            for (int hh = 0; hh < 2; ++hh)
#pragma unroll
                for (int l = 0; l < n; ++l) {
                    const double wt = tb.Wt[fk][hh * n + l];
                    if (wt == 0.0) continue;
                    sum += 2.0 * wt * hf * 0.25 * fmax(lm, sMl[le][(ff * 2 + hh) * n + l]);
                }
        } else {
            const int hh = fm_half(code);
#pragma unroll
            for (int j = 0; j < n; ++j) {
                const double wt = tb.Wt[j][hh * n + fk];
                if (wt == 0.0) continue;
                sum += 2.0 * wt * (2.0 * hf) * 0.25 * fmax(lm, sMl[le][(ff * 2) * n + j]);
            }
        }
        sF[le][q] = sum;
    }
    __syncthreads();
    double s = 0.0;
    if (act) {
        const double lx = sL[le][0][q], ly = sL[le][1][q];
        if (!idp) {
            s = (N + 1) * (lx * frcp(hx) + ly * frcp(hy));
        } else {
            // edges along x carry 2 |c| = w_b h_y / 2, along y w_a h_x / 2
            const double cx = 0.5 * sTw[0][b] * hy, cy = 0.5 * sTw[0][a] * hx;
            double sum = 0.0;
            if (a > 0) sum += cx * fmax(lx, sL[le][0][q - 1]);
            if (a < N) sum += cx * fmax(lx, sL[le][0][q + 1]);
            if (b > 0) sum += cy * fmax(ly, sL[le][1][q - n]);
            if (b < N) sum += cy * fmax(ly, sL[le][1][q + n]);
            if (a == 0) sum += sF[le][0 * n + b];
            if (a == N) sum += sF[le][1 * n + b];
            if (b == 0) sum += sF[le][2 * n + a];
            if (b == N) sum += sF[le][3 * n + a];
            s = sum * (4.0 * frcp(hx * hy)) * sTw[1][a] * sTw[1][b];
        }
    }
    s = wave_max(s);
    if ((tid & 63) == 0) sRed[tid >> 6] = s;
    __syncthreads();
    if (tid == 0) {
        // non-negative doubles order like their bit patterns; NaN and zero
        // maxima are left out, as fmax would
        double m = sRed[0];
#pragma unroll
        for (int w = 1; w < NW; ++w) m = fmax(m, sRed[w]);
        if (m > 0.0)
            atomicMax(A.acc + (blockIdx.x % kDtSpread) * kDtStride,
                      (unsigned long long)__double_as_longlong(m));
    }
    if (blockIdx.x == 0 && tid < kDtSpread) A.other[tid * kDtStride] = 0ull;
}

// ---------------------------------------------------------------------------
// modal indicator (k_indicator), features and the learned indicator
// (k_features).  Squared orthonormal-Legendre coefficients of a staged nodal
// quantity q[b'][a'], one thread per mode (i, j) = (a, b) of an element, in
// two sum-factorised passes through LDS:
//   r[b'][i] = sum_a' Vinv[i][a'] q[b'][a'],   m[j][i] = sum_b' Vinv[j][b'] r[b'][i]
// (n reads per thread and pass instead of n^2).
//  Hennemann indicator on rho p: energy = max of the energy fractions of the
//  highest and the second-highest mode shells, alpha = logistic with threshold
//  T = 0.5 10^(-1.8 (N+1)^(1/4)) and sharpness ln(9999), zero below 1e-3,
//  capped at 0.5.
//  Features: x- and y-shell energy fractions of rho and of p for the shells
//  N-3 .. N (16 values), one lane per feature.
// Outputs (FP32) go to the external element order through perm.
// ---------------------------------------------------------------------------
template <int N>
__device__ __forceinline__ double modal_x(const Tab<N>& tb, const double* Q, int a, int b)
{
    constexpr int n = N + 1;
    double r = 0.0;
#pragma unroll
    for (int aa = 0; aa < n; ++aa) r += tb.Vinv[a][aa] * Q[b * n + aa];
    return r;
}

template <int N>
__device__ __forceinline__ double modal_y_sq(const Tab<N>& tb, const double* Rx, int a, int b)
{
    constexpr int n = N + 1;
    double m = 0.0;
#pragma unroll
    for (int bb = 0; bb < n; ++bb) m += tb.Vinv[b][bb] * Rx[bb * n + a];
    return m * m;
}

template <int N>
__global__ __launch_bounds__(128) void k_indicator(const double* __restrict__ u, int E,
                                                   const int* __restrict__ perm, double gamma,
                                                   float* __restrict__ alpha)
{
    constexpr int n = N + 1, NN = n * n, EPB = 128 / NN;
    __shared__ double sQ[EPB][NN];
    __shared__ double sR[EPB][NN];
    const Tab<N>& tb = T<N>();
    const int tid = threadIdx.x;
    const int le = tid / NN, q = tid - le * NN, a = q % n, b = q / n;
    const int e = blockIdx.x * EPB + le;
    const bool act = tid < EPB * NN && e < E;
    if (act) {
        double w[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) w[v] = u[((size_t)e * 4 + v) * NN + q];
        sQ[le][q] = w[0] * (gamma - 1.0) * (w[3] - 0.5 * (w[1] * w[1] + w[2] * w[2]) / w[0]);
    }
    __syncthreads();
    if (act) sR[le][q] = modal_x<N>(tb, sQ[le], a, b);
    __syncthreads();
    if (act) sQ[le][q] = modal_y_sq<N>(tb, sR[le], a, b);  // sQ now holds m^2
    __syncthreads();
    if (!act || q != 0) return;
    double all = 0.0, low1 = 0.0, low2 = 0.0;
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i) {
            const double m2 = sQ[le][j * n + i];
            all += m2;
            if (i < N && j < N) low1 += m2;
            if (i < N - 1 && j < N - 1) low2 += m2;
        }
    const double en = fmax((all - low1) / all, (low1 - low2) / low1);
    const double T = 0.5 * pow(10.0, -1.8 * sqrt(sqrt((double)(N + 1))));
    const double s = log((1.0 - 1e-4) / 1e-4);
    double al = 1.0 / (1.0 + exp(-(s / T) * (en - T)));
    if (al < 1e-3) al = 0.0;
    alpha[perm[e]] = (float)fmin(al, 0.5);
}

// Features of a tile of TE elements per 256-thread block, in rounds of
// 256 / (N+1)^2 elements (one thread per node); the tile's state is loaded
// before its first round.  Each feature takes one lane: its shell sum of n
// squared modes; the 16 lanes of an element are consecutive lanes of one wave
// and form the total energy of each quantity from the x-shell sums with three
// butterfly steps.  NET = false writes the features; NET = true keeps them in
// LDS and wave 0 runs the network on the tile (the matrix-core pass of
// mlp::forward32: features rounded to FP32, then to BF16; weights staged once
// per block in LDS).
template <int N>
struct FeatGeom {
    static constexpr int NN = (N + 1) * (N + 1), CH = 256 / NN;
    static constexpr int R = (32 / CH) < 1 ? 1 : 32 / CH;  // rounds: 3 at N = 4, 2 at N = 3
    static constexpr int TE = R * CH;                       // 30 at N = 4, 32 at N = 3
};

template <int N, bool NET>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(7), amdgpu_num_vgpr(64))) void k_features(
    const double* __restrict__ u, int E, const int* __restrict__ perm, double gamma,
    const uint16_t* __restrict__ wb, float* __restrict__ out)
{
    using G = FeatGeom<N>;
    constexpr int n = N + 1, NN = G::NN, CH = G::CH, R = G::R, TE = G::TE;
    static_assert(TE <= 32 && N >= 3, "one wave of the network pass per tile; shells N-3 .. N");
    __shared__ double sQ[2][CH][NN];  // nodal values, then squared modes
    __shared__ double sR[2][CH][NN];  // x pass
    __shared__ __align__(16) float sX[NET ? 32 : 1][mlp::kNin + 4];
    __shared__ __align__(16) mlp::LdsWeights sW[1];  // not allocated when NET is false (unused)
    const Tab<N>& tb = T<N>();
    const int tid = threadIdx.x;
    const int le = tid / NN, q = tid - le * NN, a = q % n, b = q / n;
    const int fe = tid >> 4, f = tid & 15;
    // feature f of element fe: quantity f / 8 (rho, p), direction (f / 4) % 2
    // (x shells: sums over the y modes, y shells: over the x modes), shell N - 3 + f % 4
    const int fk = f >> 3, kk = N - 3 + (f & 3);
    const bool ydir = (f >> 2) & 1;
    const int e0 = blockIdx.x * TE;
    // the weights are staged first (their loads are issued before the state's);
    // the rounds' barriers order the staging before the network pass
    if (NET) mlp::stage_weights(sW[0], wb, tid, 256);
    double w[R][4];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int e = e0 + r * CH + le;
        if (tid < CH * NN && e < E) {
#pragma unroll
            for (int v = 0; v < 4; ++v) w[r][v] = u[((size_t)e * 4 + v) * NN + q];
        }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const bool act = tid < CH * NN && e0 + r * CH + le < E;
        if (act) {
            const double p = (gamma - 1.0) * (w[r][3] - 0.5 * (w[r][1] * w[r][1] + w[r][2] * w[r][2]) / w[r][0]);
            sQ[0][le][q] = w[r][0];
            sQ[1][le][q] = p;
        }
        __syncthreads();
        if (act) {
            sR[0][le][q] = modal_x<N>(tb, sQ[0][le], a, b);
            sR[1][le][q] = modal_x<N>(tb, sQ[1][le], a, b);
        }
        __syncthreads();
        if (act) {  // sQ now holds m^2
            sQ[0][le][q] = modal_y_sq<N>(tb, sR[0][le], a, b);
            sQ[1][le][q] = modal_y_sq<N>(tb, sR[1][le], a, b);
        }
        __syncthreads();
        if (fe < CH) {  // whole 16-lane groups
            const int e = e0 + r * CH + fe;
            const bool ok = e < E;
            double sh = 0.0, part = 0.0;
            if (ok) {
                const double* m2 = sQ[fk][fe];
#pragma unroll
                for (int j = 0; j < n; ++j) sh += ydir ? m2[kk * n + j] : m2[j * n + kk];
                if (!ydir) {
                    part = sh;
                    // the x shells below N - 3 (one at N = 4) enter the total by lane N - 3
                    if ((f & 3) == 0)
#pragma unroll
                        for (int c0 = 0; c0 < N - 3; ++c0)
#pragma unroll
                            for (int j = 0; j < n; ++j) part += m2[j * n + c0];
                }
            }
            part += __shfl_xor(part, 1, 64);
            part += __shfl_xor(part, 2, 64);
            part += __shfl_xor(part, 4, 64);
            const float v = ok ? (float)(sh / part) : 0.0f;
            if (!NET && ok) out[(size_t)perm[e] * 16 + f] = v;
            if (NET) sX[r * CH + fe][f] = v;
        }
        // the next round's staging overwrites sQ (and the network pass reads sX):
        // the reads and writes above are done
        if (NET || r + 1 < R) __syncthreads();
    }
    if (!NET || tid >= 64) return;
    const int c = tid & 31, hf = tid >> 5;
    float xv[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) xv[t] = c < TE ? sX[c][hf * 8 + t] : 0.0f;
    const float y = mlp::forward32(sW[0], mlp::pack_bf16x8(xv), tid);
    if (hf == 0 && c < TE && e0 + c < E) out[perm[e0 + c]] = y;
}

template <int N, bool NET>
static void launch_features(int E, const double* u, const int* perm, double gamma, const uint16_t* wb, float* out,
                            hipStream_t s)
{
    const int ntiles = (E + FeatGeom<N>::TE - 1) / FeatGeom<N>::TE;
    hipLaunchKernelGGL((k_features<N, NET>), dim3(ntiles), dim3(256), 0, s, u, E, perm, gamma, wb, out);
}

int launch_indicator(int N, int E, const double* u, const int* perm, double gamma, float* alpha,
                     float* feat, hipStream_t s)
{
    if (E <= 0) return 0;
    if (N != 3 && N != 4) return -1;
    if (alpha) {
        const int EPB = 128 / ((N + 1) * (N + 1));
        const int grid = (E + EPB - 1) / EPB;
        if (N == 3) hipLaunchKernelGGL(k_indicator<3>, dim3(grid), dim3(128), 0, s, u, E, perm, gamma, alpha);
        else hipLaunchKernelGGL(k_indicator<4>, dim3(grid), dim3(128), 0, s, u, E, perm, gamma, alpha);
    }
    if (feat) {
        if (N == 3) launch_features<3, false>(E, u, perm, gamma, nullptr, feat, s);
        else launch_features<4, false>(E, u, perm, gamma, nullptr, feat, s);
    }
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_learned_indicator(int N, int E, const double* u, const int* perm, double gamma, const uint16_t* wb,
                             float* alpha, hipStream_t s)
{
    if (E <= 0) return 0;
    if (N == 3) launch_features<3, true>(E, u, perm, gamma, wb, alpha, s);
    else if (N == 4) launch_features<4, true>(E, u, perm, gamma, wb, alpha, s);
    else return -1;
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

// ---------------------------------------------------------------------------
// shock indicator of combined limiting (Sec. 3.5): the Hennemann indicator on
// the pressure, not capped, FP64, one value per element in internal order.
// One thread per node stages p, one thread per mode (i, j) forms its squared
// orthonormal-Legendre coefficient (the two passes of modal_x and modal_y_sq),
// thread 0 of the element reduces.
// ---------------------------------------------------------------------------
template <int N>
__global__ __launch_bounds__(128) void k_shock_indicator(const double* __restrict__ u, int E, double gamma,
                                                         double* __restrict__ ind)
{
    constexpr int n = N + 1, NN = n * n, EPB = 128 / NN;
    __shared__ double sP[EPB][NN];
    __shared__ double sR[EPB][NN];
    const Tab<N>& tb = T<N>();
    const int tid = threadIdx.x;
    const int le = tid / NN, q = tid - le * NN, a = q % n, b = q / n;
    const int e = blockIdx.x * EPB + le;
    const bool act = tid < EPB * NN && e < E;
    if (act) {
        double w[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) w[v] = u[((size_t)e * 4 + v) * NN + q];
        sP[le][q] = (gamma - 1.0) * (w[3] - 0.5 * (w[1] * w[1] + w[2] * w[2]) / w[0]);
    }
    __syncthreads();
    if (act) sR[le][q] = modal_x<N>(tb, sP[le], a, b);
    __syncthreads();
    if (act) sP[le][q] = modal_y_sq<N>(tb, sR[le], a, b);  // sP now holds m^2
    __syncthreads();
    if (!act || q != 0) return;
    double all = 0.0, low1 = 0.0, low2 = 0.0;
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i) {
            const double m2 = sP[le][j * n + i];
            all += m2;
            if (i < N && j < N) low1 += m2;
            if (i < N - 1 && j < N - 1) low2 += m2;
        }
    const double en = fmax((all - low1) / all, (low1 - low2) / low1);
    const double T = 0.5 * pow(10.0, -1.8 * sqrt(sqrt((double)(N + 1))));
    const double s = log((1.0 - 1e-4) / 1e-4);
    const double al = 1.0 / (1.0 + exp(-(s / T) * (en - T)));
    ind[e] = al < 1e-3 ? 0.0 : al;
}

int launch_shock_indicator(int N, const DevMesh& m, const double* u, double gamma, hipStream_t s)
{
    if (m.E <= 0) return 0;
    const int EPB = 128 / ((N + 1) * (N + 1));
    const int grid = (m.E + EPB - 1) / EPB;
    if (N == 3) hipLaunchKernelGGL(k_shock_indicator<3>, dim3(grid), dim3(128), 0, s, u, m.E, gamma, m.shock_ind);
    else if (N == 4) hipLaunchKernelGGL(k_shock_indicator<4>, dim3(grid), dim3(128), 0, s, u, m.E, gamma, m.shock_ind);
    else return -1;
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

// ---------------------------------------------------------------------------
// solution transfer between meshes (Sec. 2.4): one thread per new node.
// Children take the parent polynomial at their nodes (tensor product of the
// mortar interpolation matrices); a new parent takes the exact L2 projection
// of its four children (tensor product of the mortar projections, summed).
// ---------------------------------------------------------------------------
template <int N>
__global__ __launch_bounds__(256) void k_transfer(int E, const int* __restrict__ tkind,
                                                  const int* __restrict__ tsrc,
                                                  const double* __restrict__ uold,
                                                  double* __restrict__ unew)
{
    constexpr int n = N + 1, NN = n * n;
    const Tab<N>& tb = T<N>();
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= E * NN) return;
    const int e = i / NN, q = i - e * NN, a = q % n, b = q / n;
    const int kind = tkind[e];
    double out[4] = {0, 0, 0, 0};
    if (kind == 0) {
#pragma unroll
        for (int v = 0; v < 4; ++v) out[v] = uold[((size_t)tsrc[4 * e] * 4 + v) * NN + q];
    } else if (kind == 1) {
        const int p = tsrc[4 * e], c = tsrc[4 * e + 1], cx = c & 1, cy = c >> 1;
        const double* up = uold + (size_t)p * 4 * NN;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            double acc = 0.0;
#pragma unroll
            for (int l = 0; l < n; ++l) {
                double row = 0.0;
#pragma unroll
                for (int k = 0; k < n; ++k) row += tb.I[cx][a][k] * up[(v * n + l) * n + k];
                acc += tb.I[cy][b][l] * row;
            }
            out[v] = acc;
        }
    } else {
        for (int c = 0; c < 4; ++c) {
            const int cx = c & 1, cy = c >> 1;
            const double* uc = uold + (size_t)tsrc[4 * e + c] * 4 * NN;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                double acc = 0.0;
#pragma unroll
                for (int l = 0; l < n; ++l) {
                    double row = 0.0;
#pragma unroll
                    for (int k = 0; k < n; ++k) row += tb.P[cx][a][k] * uc[(v * n + l) * n + k];
                    acc += tb.P[cy][b][l] * row;
                }
                out[v] += acc;
            }
        }
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) unew[((size_t)e * 4 + v) * NN + q] = out[v];
}

// Zhang-Shu scaling toward the reference mean (Sec. 2.4): one wave per group
// (the four children of a refined element, or one new parent).  A troubled
// group (a node with rho < eps or p < eps) is scaled by the largest theta that
// lifts every node to rho, p >= eps (aimed at eps (1 + 2^-40)); one theta per
// group keeps the group's mass.  counts[0] limited groups, counts[1] groups
// whose mean is itself below the thresholds (theta = 0).
// every node of the group scaled by t toward ub has rho >= eps and p >= eps
// (a wave-wide answer; every lane of the wave calls it)
template <int N>
__device__ bool zs_group_ok(const double* __restrict__ unew, const int* R, int cnt, int lane,
                            const double* ub, double t, double eps, double gamma)
{
    constexpr int NN = (N + 1) * (N + 1);
    int bad = 0;
    for (int j = lane; j < cnt * NN; j += 64) {
        const double* ue = unew + (size_t)R[2 + j / NN] * 4 * NN;
        const int q = j % NN;
        double w[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) w[v] = ub[v] + t * (ue[v * NN + q] - ub[v]);
        const double p = (gamma - 1.0) * (w[3] - 0.5 * (w[1] * w[1] + w[2] * w[2]) / w[0]);
        if (!(w[0] >= eps) || !(p >= eps)) bad = 1;
    }
    return !__any(bad);
}

template <int N>
__global__ __launch_bounds__(256) void k_zhang_shu(int G, const int* __restrict__ grp,
                                                   const double* __restrict__ uold,
                                                   double* __restrict__ unew, double eps,
                                                   double gamma, unsigned long long* counts)
{
    constexpr int n = N + 1, NN = n * n;
    const Tab<N>& tb = T<N>();
    const int lane = threadIdx.x & 63;
    const int g = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (g >= G) return;  // whole waves leave together
    const int* R = grp + 6 * g;
    const int kind = R[0];
    const int cnt = kind == 1 ? 4 : 1;
    const double ig1 = 1.0 / (gamma - 1.0);
    // reference mean: the old parent (refinement) or the projected parent
    const double* ref = kind == 1 ? uold + (size_t)R[1] * 4 * NN : unew + (size_t)R[2] * 4 * NN;
    double ub[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        double s = 0.0;
        for (int q = lane; q < NN; q += 64) s += tb.w[q % n] * tb.w[q / n] * ref[v * NN + q];
        ub[v] = wave_sum(s) * 0.25;
    }
    int trouble = 0;
    double em = 0.0;  // largest |E| of the group: the rounding scale of its pressures
    for (int j = lane; j < cnt * NN; j += 64) {
        const double* ue = unew + (size_t)R[2 + j / NN] * 4 * NN;
        const int q = j % NN;
        double w[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) w[v] = ue[v * NN + q];
        const double p = (gamma - 1.0) * (w[3] - 0.5 * (w[1] * w[1] + w[2] * w[2]) / w[0]);
        if (!(w[0] >= eps) || !(p >= eps)) trouble = 1;
        em = fmax(em, fabs(w[3]));
    }
    const double emax = wave_max(em);
    if (!__any(trouble)) return;
    // density aimed at eps (1 + 2^-40); pressure in addition 2^-40 max|E| above,
    // since p = (gamma-1)(E - |m|^2/(2 rho)) is known only to a few ulps of E
    const double et = eps * kMargin;
    const double pt = et + 0x1p-40 * emax;
    const double pb = (gamma - 1.0) * (ub[3] - 0.5 * (ub[1] * ub[1] + ub[2] * ub[2]) / ub[0]);
    const bool fixable = ub[0] > et && pb > pt;
    double theta = 0.0;
    if (fixable) {
        double t = 1.0;
        for (int j = lane; j < cnt * NN; j += 64) {
            const double* ue = unew + (size_t)R[2 + j / NN] * 4 * NN;
            const int q = j % NN;
            double d[4];
#pragma unroll
            for (int v = 0; v < 4; ++v) d[v] = ue[v * NN + q] - ub[v];
            double ti = 1.0;
            if (ub[0] + d[0] < et) ti = (ub[0] - et) / (-d[0]);
            ti = fmin(ti, theta_p(ub, d, pt, ig1));
            t = fmin(t, ti);
        }
        theta = wave_min(t);
        // the quadratic's coefficients cancel at the scale rho_bar E_bar and p
        // divides that rounding by rho: where a node's density gets small the
        // factor can miss, so the scaled states are checked directly and, if
        // one fails, the factor is bisected between 0 (the mean) and theta
        if (!zs_group_ok<N>(unew, R, cnt, lane, ub, theta, eps, gamma)) {
            double lo = 0.0, hi = theta;
#pragma unroll 1
            for (int it = 0; it < 60; ++it) {
                const double mid = 0.5 * (lo + hi);
                if (zs_group_ok<N>(unew, R, cnt, lane, ub, mid, eps, gamma)) lo = mid;
                else hi = mid;
            }
            theta = lo;
        }
    }
    for (int j = lane; j < cnt * NN; j += 64) {
        double* ue = unew + (size_t)R[2 + j / NN] * 4 * NN;
        const int q = j % NN;
#pragma unroll
        for (int v = 0; v < 4; ++v) ue[v * NN + q] = ub[v] + theta * (ue[v * NN + q] - ub[v]);
    }
    if (lane == 0) {
        atomicAdd(&counts[0], 1ull);
        if (!fixable) atomicAdd(&counts[1], 1ull);
    }
}

int launch_transfer(int N, int E_new, const int* tkind, const int* tsrc, const double* uold,
                    double* unew, hipStream_t s)
{
    const int NN = (N + 1) * (N + 1);
    const int grid = (E_new * NN + 255) / 256;
    if (E_new <= 0) return 0;
    if (N == 3) hipLaunchKernelGGL(k_transfer<3>, dim3(grid), dim3(256), 0, s, E_new, tkind, tsrc, uold, unew);
    else if (N == 4) hipLaunchKernelGGL(k_transfer<4>, dim3(grid), dim3(256), 0, s, E_new, tkind, tsrc, uold, unew);
    else return -1;
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_zhang_shu(int N, int G, const int* zgrp, const double* uold, double* unew, double eps,
                     double gamma, unsigned long long* counts, hipStream_t s)
{
    if (G <= 0) return 0;
    const int grid = (G + 3) / 4;  // four waves (groups) per block
    if (N == 3)
        hipLaunchKernelGGL(k_zhang_shu<3>, dim3(grid), dim3(256), 0, s, G, zgrp, uold, unew, eps, gamma, counts);
    else if (N == 4)
        hipLaunchKernelGGL(k_zhang_shu<4>, dim3(grid), dim3(256), 0, s, G, zgrp, uold, unew, eps, gamma, counts);
    else
        return -1;
    return hipGetLastError() == hipSuccess ? 0 : -1;
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
    const double p = (g - 1.0) * (w[3] - 0.5 * (w[1] * w[1] + w[2] * w[2]) / w[0]);
    const bool ok = isfinite(w[0]) && isfinite(w[1]) && isfinite(w[2]) && isfinite(w[3]) &&
                    w[0] > 0.0 && p > 0.0;
    if (!ok) atomicMin(bad, (unsigned long long)i);
}

// dt = cfl / (the maximum over the dt kernel's accumulators), once per step:
// one wave reads the kDtSpread accumulators; the stage kernels then read the
// stored value (a per-wave reduction in every block of the first stage would
// read the kDtSpread cache lines once per wave)
__global__ __launch_bounds__(64) void k_dt_final(const unsigned long long* dtmax, double cfl, double* dt_out,
                                                 DevStats* st)
{
    const double m = wave_max(__longlong_as_double((long long)dtmax[threadIdx.x * kDtStride]));
    if (threadIdx.x == 0) {
        const double dt = cfl / m;
        *dt_out = dt;
        if (st) st->dt = dt;
    }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
template <int N>
static int stage_N(const DevMesh& m, const KernelParams& kp, const double* uin, const double* un,
                   double* uout, double a, double b, const DtSource& dt, DevStats* st, int mode,
                   hipStream_t s, bool rev = false)
{
    using G = Geo<N>;
    StageArgs A;
    A.uin = uin;
    A.un = un;
    A.uout = uout;
    A.a = a;
    A.b = b;
    A.dt = dt.dt;
    A.ind = m.shock_ind;
    A.lob = m.lob;
    A.dtmax = dt.dtmax;
    A.cfl = dt.cfl;
    A.dt_out = dt.dt_out;
    // on a large mesh dt is reduced once, by k_dt_final, and the stage reads
    // it; on a small one (fewer than kFinalMin batches) the extra launch costs
    // more than the stage's own per-wave reduction
    constexpr int kFinalMin = 16384;
    if (dt.dtmax && dt.dt_out && mode == MODE_STAGE && (m.E + G::EPB - 1) / G::EPB >= kFinalMin) {
        static_assert(kDtSpread == 64, "one wave reduces the dt accumulators");
        hipLaunchKernelGGL(k_dt_final, dim3(1), dim3(64), 0, s, dt.dtmax, dt.cfl, dt.dt_out, st);
        A.dt = dt.dt_out;
        A.dtmax = nullptr;
    }
    A.fnbr = m.fnbr;
    A.fnbr2 = m.fnbr2;
    A.fmort = m.fmort;
    A.bkind = m.bkind;
    A.bext = m.bext;
    A.mort = m.mort;
    A.h = m.h;
    A.slot = m.slot;
    A.blist = m.blist;
    A.E = m.E;
    A.gamma = kp.gamma;
    A.ig1 = 1.0 / (kp.gamma - 1.0);
    A.rev = 0;
    A.beta = kp.beta;
    A.limiter = kp.limiter;
    A.vflux = kp.vflux;
    A.st = st;
    const int nb = (m.E + G::EPB - 1) / G::EPB;
    const bool mixed = kp.precision == DGIDP_MIXED;
    const int lk = kp.limiter == DGIDP_LIMIT_LOCAL ? 1
                   : kp.limiter == DGIDP_LIMIT_COMBINED ? 2
                   : kp.limiter == DGIDP_LIMIT_LOCAL_LOWORDER ? 3 : 0;
    // Positivity limiting on a large mesh: the batches with a mortar element
    // (the first m.nbm entries of the batch list) in one launch, the others in
    // a second one without mortar code (four waves per SIMD instead of three).
    // The mortar launch ends with a partly idle GPU, so a mesh of fewer than
    // kSplitMin batches, or with a larger mortar share, runs as one launch of
    // the mortar variant; so do the local-limiting modes, whose conforming
    // variant keeps three waves per SIMD.  A mesh without mortars runs the
    // conforming variant alone.
    constexpr int kSplitMin = 16384;
    const bool split = m.nbm == 0 || (lk == 0 && nb >= kSplitMin && 8LL * m.nbm <= nb);
    auto go = [&](auto modec, auto mixc, auto lkc) {
        constexpr int MD = decltype(modec)::value, LK = decltype(lkc)::value;
        constexpr bool MX = decltype(mixc)::value;
        if (!split) {
            A.blist = nullptr;  // element batches in mesh order
            A.boff = 0;
            hipLaunchKernelGGL((k_stage<N, MD, MX, LK, true>), dim3(nb), dim3(G::BS), 0, s, A);
            return;
        }
        A.blist = m.nbm > 0 ? m.blist : nullptr;
        if (m.nbm > 0) {
            A.boff = 0;
            hipLaunchKernelGGL((k_stage<N, MD, MX, LK, true>), dim3(m.nbm), dim3(G::BS), 0, s, A);
        }
        if (nb > m.nbm) {
            // (only this launch may walk its ranges backwards: its blocks cost
            // alike, where the mortar launch and an unsplit stage start the
            // costlier mortar batches first on purpose)
            A.boff = m.nbm;
            A.rev = rev ? 1 : 0;
            hipLaunchKernelGGL((k_stage<N, MD, MX, LK, false>), dim3(nb - m.nbm), dim3(G::BS), 0, s, A);
        }
    };
    using I0 = std::integral_constant<int, 0>;
    using BT = std::true_type;
    using BF = std::false_type;
    if (mode == MODE_STAGE) {
        using MS = std::integral_constant<int, MODE_STAGE>;
        if (lk == 3) {
            if (mixed) go(MS(), BT(), std::integral_constant<int, 3>());
            else go(MS(), BF(), std::integral_constant<int, 3>());
        } else if (lk == 1) {
            if (mixed) go(MS(), BT(), std::integral_constant<int, 1>());
            else go(MS(), BF(), std::integral_constant<int, 1>());
        } else if (lk == 2) {
            if (mixed) go(MS(), BT(), std::integral_constant<int, 2>());
            else go(MS(), BF(), std::integral_constant<int, 2>());
        } else {
            if (mixed) go(MS(), BT(), I0());
            else go(MS(), BF(), I0());
        }
    } else if (mode == MODE_RHS_HIGH) {
        using MH = std::integral_constant<int, MODE_RHS_HIGH>;
        if (mixed) go(MH(), BT(), I0());
        else go(MH(), BF(), I0());
    } else {
        go(std::integral_constant<int, MODE_RHS_LOW>(), BF(), I0());
    }
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_stage(int N, const DevMesh& m, const KernelParams& kp, const double* uin,
                 const double* un, double* uout, double a, double b, const DtSource& dt,
                 DevStats* st, hipStream_t s, bool rev)
{
    if (m.E == 0) return 0;
    if (N == 3) return stage_N<3>(m, kp, uin, un, uout, a, b, dt, st, MODE_STAGE, s, rev);
    if (N == 4) return stage_N<4>(m, kp, uin, un, uout, a, b, dt, st, MODE_STAGE, s, rev);
    return -1;
}

int launch_rhs(int N, const DevMesh& m, const KernelParams& kp, const double* u, int which,
               double* du, hipStream_t s)
{
    if (m.E == 0) return 0;
    const int mode = which == DGIDP_RHS_HIGH ? MODE_RHS_HIGH : MODE_RHS_LOW;
    const DtSource none;
    if (N == 3) return stage_N<3>(m, kp, u, nullptr, du, 0.0, 1.0, none, nullptr, mode, s);
    if (N == 4) return stage_N<4>(m, kp, u, nullptr, du, 0.0, 1.0, none, nullptr, mode, s);
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

int launch_dt(int N, const DevMesh& m, const KernelParams& kp, const double* u, int mode,
              unsigned long long* acc, unsigned long long* other, hipStream_t s)
{
    DtArgs A;
    A.u = u;
    A.fnbr = m.fnbr;
    A.fnbr2 = m.fnbr2;
    A.fmort = m.fmort;
    A.bkind = m.bkind;
    A.bext = m.bext;
    A.mort = m.mort;
    A.h = m.h;
    A.E = m.E;
    A.gamma = kp.gamma;
    A.mode = mode;
    A.acc = acc;
    A.other = other;
    if (N == 3)
        hipLaunchKernelGGL(k_dt<3>, dim3((m.E + DtGeo<3>::EPB - 1) / DtGeo<3>::EPB), dim3(kDtBlock), 0, s, A);
    else if (N == 4)
        hipLaunchKernelGGL(k_dt<4>, dim3((m.E + DtGeo<4>::EPB - 1) / DtGeo<4>::EPB), dim3(kDtBlock), 0, s, A);
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
