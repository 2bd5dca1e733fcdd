// Host side of dgidp: context, quadtree mesh and connectivity, state transfer,
// and the C-ABI entry points declared in include/dgidp.h.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <string>
#include <unordered_map>
#include <vector>

#include "dgidp_internal.h"
#include "dgidp_leaves.h"
#include "dgidp_par.h"

namespace dgidp {
int build_and_upload_tables(int N, std::vector<double>* nodes);
int host_tables(int N, double* out);
}  // namespace dgidp

using namespace dgidp;

// Device buffers of a context that live from one mesh to the next: a mesh
// upload or adaptation reallocates a buffer only when it needs more than the
// buffer holds (then with 25% headroom), instead of freeing and allocating
// every array each time.  The state alternates between two slots so that an
// adaptation can read the old state while it writes the new one.
enum PoolSlot {
    P_FNBR, P_FNBR2, P_FMORT, P_MORT, P_H, P_SNODE, P_SPART, P_PERM, P_BKIND, P_BEXT, P_SLOT, P_BLIST,
    P_SHOCK, P_DLO, P_LOB, P_LSV, P_U0, P_U1, P_W1, P_W2, P_TKIND, P_TSRC, P_TGRP, P_TCOUNT,
    P_COUNT
};
struct PoolBuf {
    void* p = nullptr;
    size_t cap = 0;
};

struct dgidp_ctx {
    dgidp_params p{};
    hipStream_t stream = nullptr;
    std::string err;
    std::vector<double> xi;  // LGL nodes
    // mesh (host)
    int64_t E = 0, M = 0;
    std::vector<int8_t> level;
    std::vector<int32_t> ix, iy;
    std::vector<int> perm;  // internal -> external
    double x0 = 0, y0 = 0, Lx = 1, Ly = 1;
    int nx0 = 1, ny0 = 1;
    std::vector<double> hh;  // internal [E*2]
    // device
    DevMesh dm;
    double *U = nullptr, *W1 = nullptr, *W2 = nullptr;
    double* dt_dev = nullptr;
    // two dt accumulators used in turn: the dt kernel fills one and clears the other
    unsigned long long* acc = nullptr;
    int acc_slot = 0;
    DevStats* stats = nullptr;
    unsigned long long* bad = nullptr;
    MlpState* mlp = nullptr;       // learned indicator, created on first use
    // enqueue-only SSP-RK3 steps may replay a captured graph, one per dt
    // accumulator; off by default (measured slower than direct launches here)
    bool use_graphs = false;
    hipStream_t cap = nullptr;     // capture stream
    hipGraphExec_t gexec[2] = {nullptr, nullptr};
    double gcfl[2] = {0.0, 0.0};
    float* ind_buf = nullptr;      // [E] indicator / [E*16] features staging
    size_t ind_cap = 0;
    bool has_state = false;
    // domain sides (x-, x+, y-, y+): condition and exterior state
    int bc[4] = {0, 0, 0, 0};
    double bc_ext[16] = {};
    PoolBuf pool[P_COUNT];
    int u_slot = 0;  // P_U0 + u_slot holds the state
    int64_t NB = 0;  // boundary nodes of the mesh
    std::vector<int> bface_elem;  // [NB / (N+1)] external element * 4 + face
};

namespace {

int fail(dgidp_ctx* c, int code, const std::string& msg)
{
    if (c) c->err = msg;
    return code;
}

#define HIPCHK(call)                                                                   \
    do {                                                                               \
        hipError_t _e = (call);                                                        \
        if (_e != hipSuccess)                                                          \
            return fail(ctx, DGIDP_E_DEVICE, std::string(#call) + ": " + hipGetErrorString(_e)); \
    } while (0)

template <typename T>
void dfree(T*& p)
{
    if (p) (void)hipFree(p);
    p = nullptr;
}

void drop_graphs(dgidp_ctx* c)
{
    for (int i = 0; i < 2; ++i) {
        if (c->gexec[i]) (void)hipGraphExecDestroy(c->gexec[i]);
        c->gexec[i] = nullptr;
    }
}

// a pool buffer of at least bytes (its previous contents are not kept when it
// grows); the caller has made sure that no queued work still uses it
template <typename T>
int pool_get(dgidp_ctx* c, int slot, size_t bytes, T*& out)
{
    bytes = std::max<size_t>(bytes, 1);
    PoolBuf& b = c->pool[slot];
    if (b.cap < bytes) {
        if (b.p) (void)hipFree(b.p);
        b.p = nullptr;
        b.cap = 0;
        const size_t want = bytes + bytes / 4;
        if (hipMalloc(&b.p, want) != hipSuccess) {
            b.p = nullptr;
            out = nullptr;
            return fail(c, DGIDP_E_DEVICE, "device allocation failed");
        }
        b.cap = want;
    }
    out = (T*)b.p;
    return 0;
}

void free_pool(dgidp_ctx* c)
{
    for (auto& b : c->pool) {
        if (b.p) (void)hipFree(b.p);
        b = PoolBuf();
    }
}

// forget the mesh; its device buffers stay in the pool
void free_mesh(dgidp_ctx* c)
{
    drop_graphs(c);
    c->U = c->W1 = c->W2 = nullptr;
    c->dm = DevMesh();
    c->E = c->M = 0;
    c->NB = 0;
    c->bface_elem.clear();
    c->has_state = false;
}

template <typename T>
int upload(dgidp_ctx* ctx, int slot, T*& dst, const std::vector<T>& src)
{
    const size_t bytes = std::max<size_t>(1, src.size()) * sizeof(T);
    if (int rc = pool_get(ctx, slot, bytes, dst)) return rc;
    if (!src.empty()) HIPCHK(hipMemcpy(dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice));
    return 0;
}

inline uint64_t key_of(int l, int64_t i, int64_t j)
{
    return ((uint64_t)l << 56) | ((uint64_t)i << 28) | (uint64_t)j;
}

// bits 0..30 of v moved to the even bit positions 0..60
inline uint64_t spread_bits(uint64_t v)
{
    v &= 0x7fffffffull;
    v = (v | (v << 16)) & 0x0000ffff0000ffffull;
    v = (v | (v << 8)) & 0x00ff00ff00ff00ffull;
    v = (v | (v << 4)) & 0x0f0f0f0f0f0f0f0full;
    v = (v | (v << 2)) & 0x3333333333333333ull;
    v = (v | (v << 1)) & 0x5555555555555555ull;
    return v;
}

// Morton (Z-order) key of cell (x, y): the bits of x and y interleaved, x first
inline uint64_t morton(uint64_t x, uint64_t y) { return spread_bits(x) | (spread_bits(y) << 1); }

double host_pressure(const double* u, double g)
{
    return (g - 1.0) * (u[3] - 0.5 * (u[1] * u[1] + u[2] * u[2]) / u[0]);
}

int sync_stats(dgidp_ctx* ctx, dgidp_stats* s, int nstages)
{
    DevStats h;
    HIPCHK(hipMemcpyAsync(&h, ctx->stats, sizeof(h), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    s->fv_inadmissible = (int64_t)h.fv_inadmissible;
    s->violations = (int64_t)h.violations;
    double tv, tm;
    std::memcpy(&tv, &h.theta_vol_min_bits, 8);
    std::memcpy(&tm, &h.theta_mort_min_bits, 8);
    s->theta_vol_min = tv;
    s->theta_mort_min = tm;
    s->alpha_vol_mean = h.nfaces ? h.alpha_vol_sum / (double)h.nfaces : 0.0;
    s->alpha_mort_mean = h.nmortars ? h.alpha_mort_sum / (double)h.nmortars : 0.0;
    s->dt = h.dt;
    (void)nstages;
    return 0;
}

// Connectivity of a quadtree mesh, in internal (Morton) element order.  A face
// on a non-periodic domain side has the code -2 - (its boundary face index) and
// the element itself as neighbour; boundary faces are numbered in external
// element order, then by face, and own the nodes [index (N+1), (index+1) (N+1)).
struct HostMesh {
    int64_t NBF = 0;                // boundary faces
    std::vector<int> bface_elem;    // [NBF] external element, face: e * 4 + f
    int M = 0;
    std::vector<int> perm;          // internal -> external
    std::vector<int> fnbr, fmort;   // [E*4]
    std::vector<int> fnbr2;         // [E*4] second small element of a large face, else -1
    std::vector<int> mort;          // [M*4] large, face, small0, small1
    std::vector<int> snode, spart;  // [M*3n]
};

int build_host_mesh(int N, int64_t E, const int8_t* level, const int32_t* ix, const int32_t* iy,
                    int nx0, int ny0, const int* bc, HostMesh& hm, std::string& err)
{
    if (N != 3 && N != 4) {
        err = "unsupported N";
        return DGIDP_E_UNSUPPORTED_N;
    }
    const int n = N + 1, NN = n * n;
    if (E <= 0 || !level || !ix || !iy || nx0 <= 0 || ny0 <= 0 || E > (int64_t)(1 << 30) / (NN * 4)) {
        err = "invalid mesh arguments";
        return DGIDP_E_INVALID_ARG;
    }
    // the loops over leaves and faces run on the host pool; each reports the
    // first offending index, as a serial loop would
    std::mutex red;
    constexpr int64_t kNone = INT64_MAX;
    double area = 0.0;
    int lmax = 0;
    int64_t bad = kNone;
    par_for(E, [&](int64_t lo, int64_t hi) {
        double a = 0.0;
        int lm = 0;
        int64_t b = kNone;
        for (int64_t e = lo; e < hi; ++e) {
            const int l = level[e];
            if (l < 0 || l > 20 || ix[e] < 0 || iy[e] < 0 || ix[e] >= ((int64_t)nx0 << l) ||
                iy[e] >= ((int64_t)ny0 << l)) {
                b = e;
                break;
            }
            a += std::ldexp(1.0, -2 * l);
            lm = std::max(lm, l);
        }
        std::lock_guard<std::mutex> g(red);
        area += a;  // (the tiling test below allows for the summation order)
        lmax = std::max(lmax, lm);
        bad = std::min(bad, b);
    });
    if (bad != kNone) {
        err = "leaf " + std::to_string(bad) + " outside the root grid";
        return DGIDP_E_MESH_GAP_OR_OVERLAP;
    }
    LeafLookup find;
    const int64_t dup = find.build(E, level, ix, iy, nx0, ny0);
    if (dup >= 0) {
        err = "duplicate leaf " + std::to_string(dup);
        return DGIDP_E_MESH_GAP_OR_OVERLAP;
    }
    par_for(E, [&](int64_t lo, int64_t hi) {
        int64_t b = kNone;
        for (int64_t e = lo; e < hi && b == kNone; ++e) {
            int64_t cx = ix[e], cy = iy[e];
            for (int l = level[e] - 1; l >= 0; --l) {
                cx >>= 1;
                cy >>= 1;
                if (find.get(l, cx, cy) >= 0) {
                    b = e;
                    break;
                }
            }
        }
        std::lock_guard<std::mutex> g(red);
        bad = std::min(bad, b);
    });
    if (bad != kNone) {
        err = "leaf " + std::to_string(bad) + " overlaps a coarser leaf";
        return DGIDP_E_MESH_GAP_OR_OVERLAP;
    }
    if (std::fabs(area - (double)nx0 * ny0) > 1e-9 * nx0 * ny0) {
        err = "leaves do not tile the domain";
        return DGIDP_E_MESH_GAP_OR_OVERLAP;
    }
    auto lookup = [&](int l, int64_t i, int64_t j) -> int { return (int)find.get_wrapped(l, i, j); };
    // a face of leaf e on a non-periodic side of the domain
    const bool open_x = bc && bc[0] != DGIDP_BC_PERIODIC, open_y = bc && bc[2] != DGIDP_BC_PERIODIC;
    auto on_boundary = [&](int64_t e, int f) -> bool {
        const int l = level[e];
        if (f < 2) return open_x && (f == 0 ? ix[e] == 0 : ix[e] == ((int64_t)nx0 << l) - 1);
        return open_y && (f == 2 ? iy[e] == 0 : iy[e] == ((int64_t)ny0 << l) - 1);
    };
    std::vector<int> bface((size_t)E * 4, -1);
    hm.bface_elem.clear();
    for (int64_t e = 0; e < E; ++e)
        for (int f = 0; f < 4; ++f)
            if (on_boundary(e, f)) {
                bface[e * 4 + f] = (int)hm.bface_elem.size();
                hm.bface_elem.push_back((int)(e * 4 + f));
            }
    hm.NBF = (int64_t)hm.bface_elem.size();
    // the same-level leaf across each face (-1: none, the face is nonconforming;
    // unused on boundary faces), looked up once for the ordering and pass 1
    std::vector<int> same((size_t)E * 4, -1);
    par_for(E, [&](int64_t lo, int64_t hi) {
        for (int64_t e = lo; e < hi; ++e)
            for (int f = 0; f < 4; ++f) {
                if (bface[e * 4 + f] >= 0) continue;
                const int dx = f == 0 ? -1 : (f == 1 ? 1 : 0), dy = f == 2 ? -1 : (f == 3 ? 1 : 0);
                same[e * 4 + f] = lookup(level[e], (int64_t)ix[e] + dx, (int64_t)iy[e] + dy);
            }
    });
    // internal order: Morton order of the leaves on the finest grid, cut into
    // the eight contiguous ranges that the stage kernel hands to the eight
    // XCDs; inside each range the leaves that are the small side of a mortar
    // come first, then those that are a large side, then the others.  A wave
    // then holds either mortar elements (with their longer surface work) or
    // none, mostly of one side, and the longer waves start first on each XCD
    // instead of ending the launch late.
    // role: 0 small side only, 1 large side, 2 no nonconforming face
    std::vector<int8_t> role((size_t)E, 2);
    par_for(E, [&](int64_t lo, int64_t hi) {
        for (int64_t e = lo; e < hi; ++e)
            for (int f = 0; f < 4; ++f) {
                if (bface[e * 4 + f] >= 0 || same[e * 4 + f] >= 0) continue;
                // two finer leaves across the face: a large side
                const int64_t cx = f == 0 ? 2 * (int64_t)ix[e] - 1 : f == 1 ? 2 * (int64_t)ix[e] + 2 : 2 * (int64_t)ix[e];
                const int64_t cy = f == 2 ? 2 * (int64_t)iy[e] - 1 : f == 3 ? 2 * (int64_t)iy[e] + 2 : 2 * (int64_t)iy[e];
                if (lookup(level[e] + 1, cx, cy) >= 0) role[e] = 1;
                else if (role[e] == 2) role[e] = 0;
            }
    });
    std::vector<std::pair<uint64_t, int>> ord((size_t)E);
    par_for(E, [&](int64_t lo, int64_t hi) {
        for (int64_t e = lo; e < hi; ++e) {
            const int s = lmax - level[e];
            ord[e] = {morton((uint64_t)ix[e] << s, (uint64_t)iy[e] << s), (int)e};
        }
    });
    // (the keys are distinct: chunk sorts merged give the serial order)
    par_sort(ord);
    {
        const int64_t epb = stage_block_elems(N);
        const int64_t nb = (E + epb - 1) / epb, q = nb >> 3, r = nb & 7;
        par_for(8, [&](int64_t x0, int64_t x1) {
            for (int64_t x = x0; x < x1; ++x) {
                const int64_t g0 = x * q + std::min<int64_t>(x, r), gn = q + (x < r ? 1 : 0);
                const int64_t lo = std::min<int64_t>(E, g0 * epb), hi = std::min<int64_t>(E, (g0 + gn) * epb);
                std::stable_sort(ord.begin() + lo, ord.begin() + hi,
                                 [&](const std::pair<uint64_t, int>& p1, const std::pair<uint64_t, int>& p2) {
                                     return role[p1.second] < role[p2.second];
                                 });
            }
        }, 1);
    }
    std::vector<int> inv(E);
    hm.perm.assign(E, 0);
    par_for(E, [&](int64_t lo, int64_t hi) {
        for (int64_t i = lo; i < hi; ++i) {
            hm.perm[i] = ord[i].second;
            inv[ord[i].second] = (int)i;
        }
    });
    hm.fnbr.assign(E * 4, -1);
    hm.fnbr2.assign(E * 4, -1);
    hm.fmort.assign(E * 4, -1);
    hm.mort.clear();
    int M = 0;
    // pass 1: conforming and boundary faces, and the large sides of mortars
    // (their two small neighbours; numbered below in internal order)
    std::vector<char> large((size_t)E * 4, 0);
    par_for(E, [&](int64_t lo, int64_t hi) {
        int64_t b = kNone;
        for (int64_t i = lo; i < hi; ++i) {
            const int e = hm.perm[i], l = level[e];
            for (int f = 0; f < 4; ++f) {
                if (bface[e * 4 + f] >= 0) {
                    hm.fnbr[i * 4 + f] = (int)i;
                    hm.fmort[i * 4 + f] = -2 - bface[e * 4 + f];
                    continue;
                }
                const int dx = f == 0 ? -1 : (f == 1 ? 1 : 0), dy = f == 2 ? -1 : (f == 3 ? 1 : 0);
                const int64_t cx = ix[e] + dx, cy = iy[e] + dy;
                const int g = same[e * 4 + f];
                if (g >= 0) {
                    hm.fnbr[i * 4 + f] = inv[g];
                    continue;
                }
                const int64_t nx = (int64_t)nx0 << l, ny = (int64_t)ny0 << l;
                const int64_t wx = ((cx % nx) + nx) % nx, wy = ((cy % ny) + ny) % ny;
                if (lookup(l - 1, wx >> 1, wy >> 1) >= 0) continue;  // small side: pass 2
                int s0, s1;
                if (f < 2) {
                    const int64_t sx = 2 * wx + (f == 0 ? 1 : 0);
                    s0 = lookup(l + 1, sx, 2 * wy);
                    s1 = lookup(l + 1, sx, 2 * wy + 1);
                } else {
                    const int64_t sy = 2 * wy + (f == 2 ? 1 : 0);
                    s0 = lookup(l + 1, 2 * wx, sy);
                    s1 = lookup(l + 1, 2 * wx + 1, sy);
                }
                if (s0 < 0 || s1 < 0) {
                    b = std::min<int64_t>(b, i * 4 + f);
                    continue;
                }
                hm.fnbr[i * 4 + f] = inv[s0];
                hm.fnbr2[i * 4 + f] = inv[s1];
                large[i * 4 + f] = 1;
            }
        }
        std::lock_guard<std::mutex> g(red);
        bad = std::min(bad, b);
    });
    if (bad != kNone) {
        err = "leaf " + std::to_string(hm.perm[bad / 4]) + " face " + std::to_string(bad % 4) +
              " is not 2:1 balanced";
        return DGIDP_E_MESH_NOT_BALANCED;
    }
    // mortars numbered by their large side in internal order: counts per chunk
    // of faces, their offsets, then the entries
    {
        const int64_t nk = E * 4, nc = 64;
        std::vector<int64_t> at(nc + 1, 0);
        par_for(nc, [&](int64_t c0, int64_t c1) {
            for (int64_t c = c0; c < c1; ++c)
                for (int64_t k = nk * c / nc; k < nk * (c + 1) / nc; ++k) at[c + 1] += large[k];
        }, 1);
        for (int64_t c = 0; c < nc; ++c) at[c + 1] += at[c];
        M = (int)at[nc];
        hm.mort.resize((size_t)M * 4);
        par_for(nc, [&](int64_t c0, int64_t c1) {
            for (int64_t c = c0; c < c1; ++c) {
                int64_t S = at[c];
                for (int64_t k = nk * c / nc; k < nk * (c + 1) / nc; ++k)
                    if (large[k]) {
                        hm.fmort[k] = (int)(S << 2);
                        int* m = &hm.mort[S * 4];
                        m[0] = (int)(k / 4);
                        m[1] = (int)(k % 4);
                        m[2] = hm.fnbr[k];
                        m[3] = hm.fnbr2[k];
                        ++S;
                    }
            }
        }, 1);
    }
    // pass 2: small sides point at the large element and carry their half
    par_for(M, [&](int64_t lo, int64_t hi) {
        for (int64_t S = lo; S < hi; ++S) {
            const int L = hm.mort[S * 4], f = hm.mort[S * 4 + 1];
            for (int h = 0; h < 2; ++h) {
                const int s = hm.mort[S * 4 + 2 + h];
                hm.fnbr[s * 4 + (f ^ 1)] = L;
                hm.fmort[s * 4 + (f ^ 1)] = ((int)S << 2) | 2 | h;
            }
        }
    });
    par_for(E * 4, [&](int64_t lo, int64_t hi) {
        int64_t b = kNone;
        for (int64_t i = lo; i < hi; ++i)
            if (hm.fnbr[i] < 0) {
                b = i;
                break;
            }
        std::lock_guard<std::mutex> g(red);
        bad = std::min(bad, b);
    });
    if (bad != kNone) {
        err = "face " + std::to_string(bad % 4) + " of leaf " + std::to_string(hm.perm[bad / 4]) +
              " has no 2:1 partner";
        return DGIDP_E_MESH_NOT_BALANCED;
    }
    // mortar slots: node ids, and partners of nodes that lie on two mortars
    const int NS = 3 * n;
    hm.snode.assign((size_t)M * NS, 0);
    hm.spart.assign((size_t)M * NS, -1);
    auto fq = [&](int f, int k) { return f == 0 ? k * n : (f == 1 ? k * n + N : (f == 2 ? k : N * n + k)); };
    // first slot of each node, -1 elsewhere; the buffer persists between calls
    // (the entries used are reset below), so its pages are touched once
    static thread_local std::vector<int> first;
    if (first.size() < (size_t)E * NN) first.resize((size_t)E * NN, -1);
    for (int S = 0; S < M; ++S) {
        const int L = hm.mort[S * 4], f = hm.mort[S * 4 + 1];
        for (int j = 0; j < NS; ++j) {
            int e, ff, k;
            if (j < n) {
                e = L;
                ff = f;
                k = j;
            } else {
                e = hm.mort[S * 4 + 2 + (j - n) / n];
                ff = f ^ 1;
                k = (j - n) % n;
            }
            const int node = e * NN + fq(ff, k);
            const int sid = S * NS + j;
            hm.snode[sid] = node;
            if (first[node] < 0) {
                first[node] = sid;
            } else {
                hm.spart[sid] = first[node];
                hm.spart[first[node]] = sid;
            }
        }
    }
    for (size_t sid = 0; sid < hm.snode.size(); ++sid) first[hm.snode[sid]] = -1;
    hm.M = M;
    return 0;
}

KernelParams kparams(const dgidp_ctx* c)
{
    KernelParams k;
    k.gamma = c->p.gamma;
    k.beta = c->p.beta;
    k.limiter = c->p.limiter;
    k.precision = c->p.precision;
    k.vflux = c->p.volume_flux;
    return k;
}

DtSource stored_dt(const dgidp_ctx* c)
{
    DtSource d;
    d.dt = c->dt_dev;
    return d;
}

// one limited forward-Euler stage: uout = a un + b FE(uin), with the mesh
// arrays and per-stage buffers of dm
int stage_on(dgidp_ctx* ctx, const DevMesh& dm, const double* uin, const double* un, double* uout,
             double a, double b, DevStats* st, const DtSource& dt, bool rev = false)
{
    const KernelParams kp = kparams(ctx);
    // combined limiting weighs its factors with the indicator of the stage's input
    if (kp.limiter == DGIDP_LIMIT_COMBINED && launch_shock_indicator(ctx->p.N, dm, uin, kp.gamma, ctx->stream))
        return fail(ctx, DGIDP_E_DEVICE, "indicator kernel launch failed");
    // bounds from the low-order solution: R_LO / m of the input, then the bounds
    if (kp.limiter == DGIDP_LIMIT_LOCAL_LOWORDER &&
        (launch_rhs(ctx->p.N, dm, kp, uin, DGIDP_RHS_LOW, dm.dlo, ctx->stream) ||
         launch_lowbounds(ctx->p.N, dm, kp.gamma, uin, dm.dlo, dt, dm.lsv, dm.lob, ctx->stream)))
        return fail(ctx, DGIDP_E_DEVICE, "low-order bounds launch failed");
    if (launch_stage(ctx->p.N, dm, kp, uin, un, uout, a, b, dt, st, ctx->stream, rev))
        return fail(ctx, DGIDP_E_DEVICE, "stage kernel launch failed");
    if (launch_mortar(ctx->p.N, dm, uout, b, st, ctx->stream, kp.gamma, kp.limiter))
        return fail(ctx, DGIDP_E_DEVICE, "mortar kernel launch failed");
    return 0;
}

int stage(dgidp_ctx* ctx, const double* uin, const double* un, double* uout, double a, double b,
          DevStats* st, const DtSource& dt, bool rev = false)
{
    return stage_on(ctx, ctx->dm, uin, un, uout, a, b, st, dt, rev);
}

}  // namespace

extern "C" {

const char* dgidp_last_error(dgidp_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

int dgidp_create(const dgidp_params* p, void* stream, dgidp_ctx** out)
{
    if (!p || !out) return DGIDP_E_INVALID_ARG;
    *out = nullptr;
    if (p->N != 3 && p->N != 4) return DGIDP_E_UNSUPPORTED_N;
    if (!(p->gamma > 1.0) || !(p->beta >= 0.0 && p->beta < 1.0) ||
        (p->precision != DGIDP_FP64 && p->precision != DGIDP_MIXED) ||
        (p->dt_mode != DGIDP_DT_IDP && p->dt_mode != DGIDP_DT_LOWORDER) ||
        (p->limiter != DGIDP_LIMIT_NONE && p->limiter != DGIDP_LIMIT_POSITIVITY &&
         p->limiter != DGIDP_LIMIT_LOCAL && p->limiter != DGIDP_LIMIT_COMBINED &&
         p->limiter != DGIDP_LIMIT_LOCAL_LOWORDER) ||
        (p->volume_flux != DGIDP_FLUX_RANOCHA && p->volume_flux != DGIDP_FLUX_CHANDRASHEKAR))
        return DGIDP_E_INVALID_ARG;
    dgidp_ctx* ctx = new dgidp_ctx();
    ctx->p = *p;
    ctx->stream = (hipStream_t)stream;
    if (build_and_upload_tables(p->N, &ctx->xi)) {
        delete ctx;
        return DGIDP_E_DEVICE;
    }
    // the allocation-free step's scratch address on this device (if this
    // fails, dgidp_step_noalloc tries again on its first call here)
    (void)noalloc_scratch_setup();
    if (hipMalloc((void**)&ctx->dt_dev, sizeof(double)) != hipSuccess ||
        hipMalloc((void**)&ctx->acc, 2 * kDtWords * sizeof(unsigned long long)) != hipSuccess ||
        hipMalloc((void**)&ctx->stats, sizeof(DevStats)) != hipSuccess ||
        hipMalloc((void**)&ctx->bad, sizeof(unsigned long long)) != hipSuccess ||
        hipMemset(ctx->acc, 0, 2 * kDtWords * sizeof(unsigned long long)) != hipSuccess ||
        hipMemset(ctx->stats, 0, sizeof(DevStats)) != hipSuccess) {
        dgidp_destroy(ctx);
        return DGIDP_E_DEVICE;
    }
    *out = ctx;
    return 0;
}

void dgidp_destroy(dgidp_ctx* ctx)
{
    if (!ctx) return;
    if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
    else (void)hipDeviceSynchronize();
    free_mesh(ctx);
    free_pool(ctx);
    dfree(ctx->dt_dev);
    dfree(ctx->acc);
    dfree(ctx->ind_buf);
    if (ctx->mlp) mlp_destroy(ctx->mlp);
    if (ctx->cap) (void)hipStreamDestroy(ctx->cap);
    dfree(ctx->stats);
    dfree(ctx->bad);
    delete ctx;
}

int dgidp_set_stream(dgidp_ctx* ctx, void* stream)
{
    if (!ctx) return DGIDP_E_INVALID_ARG;
    ctx->stream = (hipStream_t)stream;
    return 0;
}

int dgidp_synchronize(dgidp_ctx* ctx)
{
    if (!ctx) return DGIDP_E_INVALID_ARG;
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return 0;
}

int dgidp_mesh_upload(dgidp_ctx* ctx, int64_t E, const int8_t* level, const int32_t* ix,
                      const int32_t* iy, double x0, double y0, double Lx, double Ly, int nx0,
                      int ny0)
{
    if (!ctx) return DGIDP_E_INVALID_ARG;
    if (!(Lx > 0) || !(Ly > 0)) return fail(ctx, DGIDP_E_INVALID_ARG, "invalid domain size");
    if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
    free_mesh(ctx);
    const int N = ctx->p.N, n = N + 1, NN = n * n;
    HostMesh hm;
    std::string err;
    const int code = build_host_mesh(N, E, level, ix, iy, nx0, ny0, ctx->bc, hm, err);
    if (code) return fail(ctx, code, err);
    // every boundary node starts with its side's condition and exterior state
    const int64_t NB = hm.NBF * n;
    std::vector<int8_t> bkind((size_t)NB);
    std::vector<double> bext((size_t)NB * 4);
    for (int64_t j = 0; j < hm.NBF; ++j) {
        const int f = hm.bface_elem[j] & 3;
        for (int k = 0; k < n; ++k) {
            bkind[j * n + k] = (int8_t)ctx->bc[f];
            for (int v = 0; v < 4; ++v) bext[(j * n + k) * 4 + v] = ctx->bc_ext[f * 4 + v];
        }
    }
    const int M = hm.M;
    int nbm = 0;
    std::vector<double> hh(E * 2);
    for (int64_t i = 0; i < E; ++i) {
        const int e = hm.perm[i], l = level[e];
        hh[2 * i] = Lx / (double)((int64_t)nx0 << l);
        hh[2 * i + 1] = Ly / (double)((int64_t)ny0 << l);
    }
    ctx->level.assign(level, level + E);
    ctx->ix.assign(ix, ix + E);
    ctx->iy.assign(iy, iy + E);
    ctx->perm = hm.perm;
    ctx->hh = hh;
    ctx->x0 = x0;
    ctx->y0 = y0;
    ctx->Lx = Lx;
    ctx->Ly = Ly;
    ctx->nx0 = nx0;
    ctx->ny0 = ny0;
    // stage-kernel batches with a mortar element first (their own launch)
    const int64_t epb = stage_block_elems(N), nbat = (E + epb - 1) / epb;
    std::vector<int> blist;
    blist.reserve((size_t)nbat);
    for (int pass = 0; pass < 2; ++pass)
        for (int64_t bt = 0; bt < nbat; ++bt) {
            bool mort = false;
            for (int64_t i = bt * epb; i < std::min(E, (bt + 1) * epb) && !mort; ++i)
                for (int f = 0; f < 4; ++f) mort = mort || hm.fmort[i * 4 + f] >= 0;
            if (mort == (pass == 0)) blist.push_back((int)bt);
            if (pass == 0 && mort) ++nbm;
        }
    int rc = 0;
    if ((rc = upload(ctx, P_FNBR, ctx->dm.fnbr, hm.fnbr)) || (rc = upload(ctx, P_FNBR2, ctx->dm.fnbr2, hm.fnbr2)) ||
        (rc = upload(ctx, P_BLIST, ctx->dm.blist, blist)) ||
        (rc = upload(ctx, P_FMORT, ctx->dm.fmort, hm.fmort)) ||
        (rc = upload(ctx, P_MORT, ctx->dm.mort, hm.mort)) || (rc = upload(ctx, P_H, ctx->dm.h, hh)) ||
        (rc = upload(ctx, P_SNODE, ctx->dm.slot_node, hm.snode)) ||
        (rc = upload(ctx, P_SPART, ctx->dm.slot_partner, hm.spart)) ||
        (rc = upload(ctx, P_PERM, ctx->dm.perm, hm.perm)) ||
        (rc = upload(ctx, P_BKIND, ctx->dm.bkind, bkind)) || (rc = upload(ctx, P_BEXT, ctx->dm.bext, bext))) {
        free_mesh(ctx);  // no half-built mesh: the context has none
        return rc;
    }
    const size_t sz = (size_t)E * 4 * NN * sizeof(double);
    if ((rc = pool_get(ctx, P_SLOT, (size_t)M * 3 * n * kSlotW * sizeof(double), ctx->dm.slot)) ||
        (rc = pool_get(ctx, P_SHOCK, (size_t)E * sizeof(double), ctx->dm.shock_ind)) ||
        (ctx->p.limiter == DGIDP_LIMIT_LOCAL_LOWORDER &&
         ((rc = pool_get(ctx, P_DLO, sz, ctx->dm.dlo)) ||
          (rc = pool_get(ctx, P_LOB, (size_t)E * 3 * NN * sizeof(double), ctx->dm.lob)) ||
          (rc = pool_get(ctx, P_LSV, (size_t)E * 2 * NN * sizeof(double), ctx->dm.lsv)))) ||
        (rc = pool_get(ctx, P_U0 + ctx->u_slot, sz, ctx->U)) || (rc = pool_get(ctx, P_W1, sz, ctx->W1)) ||
        (rc = pool_get(ctx, P_W2, sz, ctx->W2))) {
        free_mesh(ctx);
        return rc;
    }
    // every buffer is in place: only now does the context hold the mesh
    ctx->NB = NB;
    ctx->bface_elem = hm.bface_elem;
    ctx->E = E;
    ctx->M = M;
    ctx->dm.E = (int)E;
    ctx->dm.M = M;
    ctx->dm.nbm = nbm;
    return 0;
}

int dgidp_mesh_validate(int N, int64_t n_leaves, const int8_t* level, const int32_t* ix,
                        const int32_t* iy, int nx0, int ny0, int64_t* n_mortars,
                        int64_t* n_two_mortar_nodes, char* msg, int msglen)
{
    HostMesh hm;
    std::string err;
    const int code = build_host_mesh(N, n_leaves, level, ix, iy, nx0, ny0, nullptr, hm, err);
    if (msg && msglen > 0) {
        std::snprintf(msg, (size_t)msglen, "%s", err.c_str());
    }
    if (code) return code;
    if (n_mortars) *n_mortars = hm.M;
    if (n_two_mortar_nodes) {
        int64_t c = 0;
        for (int p : hm.spart) c += p >= 0;
        *n_two_mortar_nodes = c / 2;
    }
    return 0;
}

namespace {
// an exterior state must be a finite admissible state (rho > 0, p > 0)
bool admissible_state(const double* u, double gamma)
{
    for (int v = 0; v < 4; ++v)
        if (!std::isfinite(u[v])) return false;
    if (!(u[0] > 0.0)) return false;
    return (gamma - 1.0) * (u[3] - 0.5 * (u[1] * u[1] + u[2] * u[2]) / u[0]) > 0.0;
}
}  // namespace

int dgidp_set_boundaries(dgidp_ctx* ctx, const int* bc, const double* ext)
{
    if (!ctx || !bc) return DGIDP_E_INVALID_ARG;
    if (ctx->E > 0) return fail(ctx, DGIDP_E_INVALID_ARG, "set the boundaries before uploading the mesh");
    for (int f = 0; f < 4; ++f)
        if (bc[f] < DGIDP_BC_PERIODIC || bc[f] > DGIDP_BC_OUTFLOW)
            return fail(ctx, DGIDP_E_INVALID_ARG, "unknown boundary condition");
    if ((bc[0] == DGIDP_BC_PERIODIC) != (bc[1] == DGIDP_BC_PERIODIC) ||
        (bc[2] == DGIDP_BC_PERIODIC) != (bc[3] == DGIDP_BC_PERIODIC))
        return fail(ctx, DGIDP_E_INVALID_ARG, "opposite sides must both be periodic or both not");
    for (int f = 0; f < 4; ++f)
        if (bc[f] == DGIDP_BC_CHARACTERISTIC && (!ext || !admissible_state(ext + 4 * f, ctx->p.gamma)))
            return fail(ctx, DGIDP_E_INVALID_ARG, "a characteristic side needs an admissible exterior state");
    for (int f = 0; f < 4; ++f) {
        ctx->bc[f] = bc[f];
        for (int v = 0; v < 4; ++v) ctx->bc_ext[f * 4 + v] = ext ? ext[f * 4 + v] : 0.0;
    }
    return 0;
}

int dgidp_boundary_nodes(dgidp_ctx* ctx, int64_t* n_nodes, int64_t* nodes)
{
    if (!ctx || !n_nodes) return DGIDP_E_INVALID_ARG;
    if (ctx->E == 0) return fail(ctx, DGIDP_E_NO_MESH, "no mesh");
    *n_nodes = ctx->NB;
    if (nodes) {
        const int n = ctx->p.N + 1;
        for (size_t j = 0; j < ctx->bface_elem.size(); ++j)
            for (int k = 0; k < n; ++k) {
                nodes[(j * n + k) * 3 + 0] = ctx->bface_elem[j] >> 2;
                nodes[(j * n + k) * 3 + 1] = ctx->bface_elem[j] & 3;
                nodes[(j * n + k) * 3 + 2] = k;
            }
    }
    return 0;
}

int dgidp_set_boundary_states(dgidp_ctx* ctx, const int8_t* kind, const double* ext)
{
    if (!ctx || !kind || !ext) return DGIDP_E_INVALID_ARG;
    if (ctx->E == 0) return fail(ctx, DGIDP_E_NO_MESH, "no mesh");
    for (int64_t j = 0; j < ctx->NB; ++j) {
        if (kind[j] < DGIDP_BC_WALL || kind[j] > DGIDP_BC_OUTFLOW)
            return fail(ctx, DGIDP_E_INVALID_ARG, "boundary node " + std::to_string(j) + ": unknown condition");
        if (kind[j] == DGIDP_BC_CHARACTERISTIC && !admissible_state(ext + 4 * j, ctx->p.gamma))
            return fail(ctx, DGIDP_E_INVALID_ARG,
                        "boundary node " + std::to_string(j) + ": exterior state not admissible");
    }
    if (ctx->NB == 0) return 0;
    // the stream may still read the previous states
    HIPCHK(hipStreamSynchronize(ctx->stream));
    HIPCHK(hipMemcpy(ctx->dm.bkind, kind, (size_t)ctx->NB, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(ctx->dm.bext, ext, (size_t)ctx->NB * 4 * sizeof(double), hipMemcpyHostToDevice));
    return 0;
}

int dgidp_mesh_validate_bc(int N, int64_t n_leaves, const int8_t* level, const int32_t* ix,
                           const int32_t* iy, int nx0, int ny0, const int* bc, int64_t* n_mortars,
                           int64_t* n_boundary_nodes, char* msg, int msglen)
{
    std::string err;
    int code = 0;
    if (bc) {
        for (int f = 0; f < 4 && !code; ++f)
            if (bc[f] < DGIDP_BC_PERIODIC || bc[f] > DGIDP_BC_OUTFLOW) {
                err = "unknown boundary condition";
                code = DGIDP_E_INVALID_ARG;
            }
        if (!code && ((bc[0] == DGIDP_BC_PERIODIC) != (bc[1] == DGIDP_BC_PERIODIC) ||
                      (bc[2] == DGIDP_BC_PERIODIC) != (bc[3] == DGIDP_BC_PERIODIC))) {
            err = "opposite sides must both be periodic or both not";
            code = DGIDP_E_INVALID_ARG;
        }
    }
    HostMesh hm;
    if (!code) code = build_host_mesh(N, n_leaves, level, ix, iy, nx0, ny0, bc, hm, err);
    if (msg && msglen > 0) std::snprintf(msg, (size_t)msglen, "%s", err.c_str());
    if (code) return code;
    if (n_mortars) *n_mortars = hm.M;
    if (n_boundary_nodes) *n_boundary_nodes = hm.NBF * (N + 1);
    return 0;
}

int dgidp_mesh_info(dgidp_ctx* ctx, int64_t* n_elements, int64_t* n_mortars)
{
    if (!ctx) return DGIDP_E_INVALID_ARG;
    if (n_elements) *n_elements = ctx->E;
    if (n_mortars) *n_mortars = ctx->M;
    return 0;
}

int dgidp_node_coords(dgidp_ctx* ctx, double* x, double* y)
{
    if (!ctx || !x || !y) return DGIDP_E_INVALID_ARG;
    if (!ctx->E) return fail(ctx, DGIDP_E_NO_MESH, "no mesh");
    const int n = ctx->p.N + 1;
    for (int64_t e = 0; e < ctx->E; ++e) {
        const int l = ctx->level[e];
        const double hx = ctx->Lx / (double)((int64_t)ctx->nx0 << l);
        const double hy = ctx->Ly / (double)((int64_t)ctx->ny0 << l);
        for (int b = 0; b < n; ++b)
            for (int a = 0; a < n; ++a) {
                const size_t i = ((size_t)e * n + b) * n + a;
                x[i] = ctx->x0 + (ctx->ix[e] + 0.5 * (ctx->xi[a] + 1.0)) * hx;
                y[i] = ctx->y0 + (ctx->iy[e] + 0.5 * (ctx->xi[b] + 1.0)) * hy;
            }
    }
    return 0;
}

int dgidp_state_upload(dgidp_ctx* ctx, const double* u, int on_device)
{
    if (!ctx || !u) return DGIDP_E_INVALID_ARG;
    if (!ctx->E) return fail(ctx, DGIDP_E_NO_MESH, "no mesh");
    const int N = ctx->p.N, NN = (N + 1) * (N + 1);
    const size_t sz = (size_t)ctx->E * 4 * NN * sizeof(double);
    if (on_device) {
        HIPCHK(hipMemsetAsync(ctx->bad, 0xff, sizeof(unsigned long long), ctx->stream));
        if (launch_check_state(N, (int)ctx->E, ctx->p.gamma, u, ctx->bad, ctx->stream))
            return fail(ctx, DGIDP_E_DEVICE, "check kernel launch failed");
        unsigned long long bad = 0;
        HIPCHK(hipMemcpyAsync(&bad, ctx->bad, sizeof(bad), hipMemcpyDeviceToHost, ctx->stream));
        HIPCHK(hipStreamSynchronize(ctx->stream));
        if (bad != ~0ull)
            return fail(ctx, DGIDP_E_STATE_INADMISSIBLE,
                        "inadmissible state at element " + std::to_string(bad / NN) + " node " + std::to_string(bad % NN));
        if (launch_permute(N, (int)ctx->E, ctx->dm.perm, u, ctx->U, 1, ctx->stream))
            return fail(ctx, DGIDP_E_DEVICE, "permute kernel launch failed");
    } else {
        for (int64_t e = 0; e < ctx->E; ++e)
            for (int q = 0; q < NN; ++q) {
                double w[4];
                for (int v = 0; v < 4; ++v) w[v] = u[((size_t)e * 4 + v) * NN + q];
                const double p = host_pressure(w, ctx->p.gamma);
                if (!(std::isfinite(w[0]) && std::isfinite(w[1]) && std::isfinite(w[2]) &&
                      std::isfinite(w[3]) && w[0] > 0.0 && p > 0.0))
                    return fail(ctx, DGIDP_E_STATE_INADMISSIBLE,
                                "inadmissible state at element " + std::to_string(e) + " node " + std::to_string(q));
            }
        HIPCHK(hipMemcpyAsync(ctx->W1, u, sz, hipMemcpyHostToDevice, ctx->stream));
        if (launch_permute(N, (int)ctx->E, ctx->dm.perm, ctx->W1, ctx->U, 1, ctx->stream))
            return fail(ctx, DGIDP_E_DEVICE, "permute kernel launch failed");
        HIPCHK(hipStreamSynchronize(ctx->stream));
    }
    ctx->has_state = true;
    return 0;
}

static int to_external(dgidp_ctx* ctx, const double* src_int, double* dst, int on_device)
{
    const int N = ctx->p.N, NN = (N + 1) * (N + 1);
    const size_t sz = (size_t)ctx->E * 4 * NN * sizeof(double);
    if (on_device) {
        if (launch_permute(N, (int)ctx->E, ctx->dm.perm, src_int, dst, 0, ctx->stream))
            return fail(ctx, DGIDP_E_DEVICE, "permute kernel launch failed");
        return 0;
    }
    double* tmp = src_int == ctx->W2 ? ctx->W1 : ctx->W2;
    if (launch_permute(N, (int)ctx->E, ctx->dm.perm, src_int, tmp, 0, ctx->stream))
        return fail(ctx, DGIDP_E_DEVICE, "permute kernel launch failed");
    HIPCHK(hipMemcpyAsync(dst, tmp, sz, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return 0;
}

int dgidp_state_download(dgidp_ctx* ctx, double* u, int on_device)
{
    if (!ctx || !u) return DGIDP_E_INVALID_ARG;
    if (!ctx->has_state) return fail(ctx, DGIDP_E_NO_STATE, "no state");
    return to_external(ctx, ctx->U, u, on_device);
}

int dgidp_state_check(dgidp_ctx* ctx, int64_t* first_bad)
{
    if (!ctx || !first_bad) return DGIDP_E_INVALID_ARG;
    if (!ctx->has_state) return fail(ctx, DGIDP_E_NO_STATE, "no state");
    const int N = ctx->p.N, NN = (N + 1) * (N + 1);
    HIPCHK(hipMemsetAsync(ctx->bad, 0xff, sizeof(unsigned long long), ctx->stream));
    if (launch_check_state(N, (int)ctx->E, ctx->p.gamma, ctx->U, ctx->bad, ctx->stream))
        return fail(ctx, DGIDP_E_DEVICE, "check kernel launch failed");
    unsigned long long bad = 0;
    HIPCHK(hipMemcpyAsync(&bad, ctx->bad, sizeof(bad), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    *first_bad = bad == ~0ull ? -1 : (int64_t)ctx->perm[bad / NN] * NN + (int64_t)(bad % NN);
    return 0;
}

int dgidp_rhs(dgidp_ctx* ctx, int which, double* du, int on_device)
{
    if (!ctx || !du || (which != DGIDP_RHS_HIGH && which != DGIDP_RHS_LOW)) return DGIDP_E_INVALID_ARG;
    if (!ctx->has_state) return fail(ctx, DGIDP_E_NO_STATE, "no state");
    if (launch_rhs(ctx->p.N, ctx->dm, kparams(ctx), ctx->U, which, ctx->W1, ctx->stream))
        return fail(ctx, DGIDP_E_DEVICE, "rhs kernel launch failed");
    return to_external(ctx, ctx->W1, du, on_device);
}

// enqueue the dt kernel on the current state; *src tells the next stage kernel
// to take dt = cfl / max from the accumulator it fills
static int enqueue_dt(dgidp_ctx* ctx, double cfl, int mode, DtSource* src)
{
    unsigned long long* acc = ctx->acc + ctx->acc_slot * kDtWords;
    unsigned long long* other = ctx->acc + (ctx->acc_slot ^ 1) * kDtWords;
    if (launch_dt(ctx->p.N, ctx->dm, kparams(ctx), ctx->U, mode, acc, other, ctx->stream))
        return fail(ctx, DGIDP_E_DEVICE, "dt kernel launch failed");
    ctx->acc_slot ^= 1;
    src->dt = nullptr;
    src->dtmax = acc;
    src->cfl = cfl;
    src->dt_out = ctx->dt_dev;
    return 0;
}

// dt = cfl / max computed on the host from the accumulator (same IEEE division)
static int host_dt(dgidp_ctx* ctx, double cfl, int mode, double* dt)
{
    DtSource src;
    int rc = enqueue_dt(ctx, cfl, mode, &src);
    if (rc) return rc;
    std::vector<unsigned long long> bits(kDtWords);
    HIPCHK(hipMemcpyAsync(bits.data(), src.dtmax, kDtWords * sizeof(unsigned long long),
                          hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    double m = 0.0;
    for (int i = 0; i < kDtSpread; ++i) {
        double v;
        std::memcpy(&v, &bits[(size_t)i * kDtStride], sizeof(v));
        m = std::max(m, v);
    }
    *dt = cfl / m;
    return 0;
}

int dgidp_max_dt(dgidp_ctx* ctx, double cfl, double* dt)
{
    if (!ctx || !dt || !(cfl > 0)) return DGIDP_E_INVALID_ARG;
    if (!ctx->has_state) return fail(ctx, DGIDP_E_NO_STATE, "no state");
    return host_dt(ctx, cfl, ctx->p.dt_mode, dt);
}

int dgidp_limit(dgidp_ctx* ctx, double dt, dgidp_stats* s)
{
    if (!ctx || !(dt > 0)) return DGIDP_E_INVALID_ARG;
    if (!ctx->has_state) return fail(ctx, DGIDP_E_NO_STATE, "no state");
    if (ctx->p.strict_dt) {
        double bound = 0;
        int rc = host_dt(ctx, 1.0, DGIDP_DT_IDP, &bound);
        if (rc) return rc;
        if (dt > bound)
            return fail(ctx, DGIDP_E_DT, "dt above the IDP bound " + std::to_string(bound));
    }
    if (launch_set_double(ctx->dt_dev, dt, ctx->stream)) return fail(ctx, DGIDP_E_DEVICE, "launch failed");
    DevStats* st = s ? ctx->stats : nullptr;
    if (st && launch_stats_reset(st, ctx->stream)) return fail(ctx, DGIDP_E_DEVICE, "launch failed");
    int rc = stage(ctx, ctx->U, nullptr, ctx->W1, 0.0, 1.0, st, stored_dt(ctx));
    if (rc) return rc;
    std::swap(ctx->U, ctx->W1);
    // captured steps hold the old state and stage buffer addresses
    drop_graphs(ctx);
    if (s) {
        rc = sync_stats(ctx, s, 1);
        s->dt = dt;
        return rc;
    }
    return 0;
}

// the three stages; the first takes dt from first_dt, the others from the
// stored value (which the first stage writes when it computes dt itself)
static int ssprk3(dgidp_ctx* ctx, dgidp_stats* s, const DtSource& first_dt)
{
    DevStats* st = s ? ctx->stats : nullptr;
    const DtSource dt = stored_dt(ctx);
    int rc;
    if ((rc = stage(ctx, ctx->U, nullptr, ctx->W1, 0.0, 1.0, st, first_dt))) return rc;
    if ((rc = stage(ctx, ctx->W1, ctx->U, ctx->W2, 0.75, 0.25, st, dt, true))) return rc;
    if ((rc = stage(ctx, ctx->W2, ctx->U, ctx->U, 1.0 / 3.0, 2.0 / 3.0, st, dt))) return rc;
    return 0;
}

// record one enqueue-only step (dt kernel and three stages) for accumulator
// slot `slot` into a graph; nothing runs during the capture
static int capture_step(dgidp_ctx* ctx, double cfl, int slot)
{
    if (!ctx->cap && hipStreamCreateWithFlags(&ctx->cap, hipStreamNonBlocking) != hipSuccess) {
        ctx->cap = nullptr;
        return -1;
    }
    if (ctx->gexec[slot]) (void)hipGraphExecDestroy(ctx->gexec[slot]);
    ctx->gexec[slot] = nullptr;
    hipStream_t keep = ctx->stream;
    ctx->stream = ctx->cap;
    ctx->acc_slot = slot;
    int rc = hipStreamBeginCapture(ctx->cap, hipStreamCaptureModeThreadLocal) == hipSuccess ? 0 : -1;
    if (!rc) {
        DtSource src;
        rc = enqueue_dt(ctx, cfl, ctx->p.dt_mode, &src);
        if (!rc) rc = ssprk3(ctx, nullptr, src);
        hipGraph_t g = nullptr;
        const hipError_t e = hipStreamEndCapture(ctx->cap, &g);
        if (!rc && e == hipSuccess && g &&
            hipGraphInstantiate(&ctx->gexec[slot], g, nullptr, nullptr, 0) == hipSuccess)
            ctx->gcfl[slot] = cfl;
        else
            rc = -1;
        if (g) (void)hipGraphDestroy(g);
    }
    ctx->stream = keep;
    ctx->acc_slot = slot;
    if (rc) {
        ctx->gexec[slot] = nullptr;
        (void)hipGetLastError();
    }
    return rc;
}

int dgidp_set_graphs(dgidp_ctx* ctx, int enable)
{
    if (!ctx) return DGIDP_E_INVALID_ARG;
    ctx->use_graphs = enable != 0;
    if (!ctx->use_graphs) drop_graphs(ctx);
    return 0;
}

int dgidp_step(dgidp_ctx* ctx, double cfl, double* dt_used, dgidp_stats* s)
{
    if (!ctx || !(cfl > 0)) return DGIDP_E_INVALID_ARG;
    if (!ctx->has_state) return fail(ctx, DGIDP_E_NO_STATE, "no state");
    if (!dt_used && !s && ctx->use_graphs) {
        const int slot = ctx->acc_slot;
        if ((ctx->gexec[slot] && ctx->gcfl[slot] == cfl) || capture_step(ctx, cfl, slot) == 0) {
            HIPCHK(hipGraphLaunch(ctx->gexec[slot], ctx->stream));
            ctx->acc_slot ^= 1;
            return 0;
        }
        ctx->use_graphs = false;  // capture not available: launch kernel by kernel
    }
    DevStats* st = s ? ctx->stats : nullptr;
    if (st && launch_stats_reset(st, ctx->stream)) return fail(ctx, DGIDP_E_DEVICE, "launch failed");
    DtSource src;
    int rc = enqueue_dt(ctx, cfl, ctx->p.dt_mode, &src);
    if (rc) return rc;
    if ((rc = ssprk3(ctx, s, src))) return rc;
    if (dt_used) {
        HIPCHK(hipMemcpyAsync(dt_used, ctx->dt_dev, sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
        HIPCHK(hipStreamSynchronize(ctx->stream));
    }
    if (s) return sync_stats(ctx, s, 3);
    return 0;
}

int dgidp_step_dt(dgidp_ctx* ctx, double dt, dgidp_stats* s)
{
    if (!ctx || !(dt > 0)) return DGIDP_E_INVALID_ARG;
    if (!ctx->has_state) return fail(ctx, DGIDP_E_NO_STATE, "no state");
    if (launch_set_double(ctx->dt_dev, dt, ctx->stream)) return fail(ctx, DGIDP_E_DEVICE, "launch failed");
    DevStats* st = s ? ctx->stats : nullptr;
    if (st && launch_stats_reset(st, ctx->stream)) return fail(ctx, DGIDP_E_DEVICE, "launch failed");
    int rc = ssprk3(ctx, s, stored_dt(ctx));
    if (rc) return rc;
    if (s) {
        rc = sync_stats(ctx, s, 3);
        s->dt = dt;
        return rc;
    }
    return 0;
}

int dgidp_step_noalloc(dgidp_ctx* ctx, double cfl)
{
    if (!ctx || !(cfl > 0)) return DGIDP_E_INVALID_ARG;
    if (!ctx->has_state) return fail(ctx, DGIDP_E_NO_STATE, "no state");
    size_t cap = 0;
    char* base = (char*)noalloc_scratch(&cap);
    if (!base && noalloc_scratch_setup() == 0) base = (char*)noalloc_scratch(&cap);
    if (!base) return fail(ctx, DGIDP_E_DEVICE, "scratch address not available on this device");
    // carve the per-step buffers from the scratch array, 256-byte aligned
    const int N = ctx->p.N, n = N + 1, NN = n * n;
    const size_t E = (size_t)ctx->E, M = (size_t)ctx->M;
    const size_t state = E * 4 * NN * sizeof(double);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t at = off;
        off += (std::max<size_t>(bytes, 1) + 255) & ~size_t(255);
        return at;
    };
    const size_t o_acc = take(2 * kDtWords * sizeof(unsigned long long));
    const size_t o_dt = take(sizeof(double));
    const size_t o_w1 = take(state), o_w2 = take(state);
    const size_t o_slot = take(M * 3 * n * kSlotW * sizeof(double));
    const size_t o_ind = take(E * sizeof(double));
    size_t o_dlo = 0, o_lob = 0, o_lsv = 0;
    if (ctx->p.limiter == DGIDP_LIMIT_LOCAL_LOWORDER) {
        o_dlo = take(state);
        o_lob = take(E * 3 * NN * sizeof(double));
        o_lsv = take(E * 2 * NN * sizeof(double));
    }
    if (off > cap)
        return fail(ctx, DGIDP_E_INVALID_ARG,
                    "dgidp_step_noalloc: this mesh needs " + std::to_string(off) +
                        " bytes of scratch, the maximum is " + std::to_string(cap));
    DevMesh dm = ctx->dm;
    dm.slot = (double*)(base + o_slot);
    dm.shock_ind = (double*)(base + o_ind);
    if (ctx->p.limiter == DGIDP_LIMIT_LOCAL_LOWORDER) {
        dm.dlo = (double*)(base + o_dlo);
        dm.lob = (double*)(base + o_lob);
        dm.lsv = (double*)(base + o_lsv);
    }
    unsigned long long* acc = (unsigned long long*)(base + o_acc);
    double* dtp = (double*)(base + o_dt);
    double* W1 = (double*)(base + o_w1);
    double* W2 = (double*)(base + o_w2);
    // the array keeps the previous call's contents: the dt maxima must start at 0
    if (launch_fill_u64(acc, 2 * kDtWords, 0ull, ctx->stream) ||
        launch_dt(N, dm, kparams(ctx), ctx->U, ctx->p.dt_mode, acc, acc + kDtWords, ctx->stream))
        return fail(ctx, DGIDP_E_DEVICE, "dt launch failed");
    DtSource first;
    first.dtmax = acc;
    first.cfl = cfl;
    first.dt_out = dtp;
    DtSource stored;
    stored.dt = dtp;
    int rc;
    if ((rc = stage_on(ctx, dm, ctx->U, nullptr, W1, 0.0, 1.0, nullptr, first)) ||
        (rc = stage_on(ctx, dm, W1, ctx->U, W2, 0.75, 0.25, nullptr, stored, true)) ||
        (rc = stage_on(ctx, dm, W2, ctx->U, ctx->U, 1.0 / 3.0, 2.0 / 3.0, nullptr, stored)))
        return rc;
    return 0;
}

int dgidp_time_kernels(dgidp_ctx* ctx, int reps, double* ms)
{
    if (!ctx || !ms || reps <= 0) return DGIDP_E_INVALID_ARG;
    if (!ctx->has_state) return fail(ctx, DGIDP_E_NO_STATE, "no state");
    const KernelParams kp = kparams(ctx);
    hipEvent_t ev[6];
    for (auto& e : ev) HIPCHK(hipEventCreate(&e));
    // the three stage configurations on the current state: U -> W1 (a = 0),
    // then (W1, U) -> W2 and (W2, U) -> W1 with u^n = U; U is only read
    double dt = 0.0;
    int rc = host_dt(ctx, 0.5, ctx->p.dt_mode, &dt);
    if (rc) return rc;
    if (launch_set_double(ctx->dt_dev, dt, ctx->stream)) return fail(ctx, DGIDP_E_DEVICE, "launch failed");
    if (kp.limiter == DGIDP_LIMIT_COMBINED &&
        launch_shock_indicator(ctx->p.N, ctx->dm, ctx->U, kp.gamma, ctx->stream))
        return fail(ctx, DGIDP_E_DEVICE, "indicator kernel launch failed");
    // (the low-order-solution bounds are formed once, outside the timed stages)
    if (kp.limiter == DGIDP_LIMIT_LOCAL_LOWORDER &&
        (launch_rhs(ctx->p.N, ctx->dm, kp, ctx->U, DGIDP_RHS_LOW, ctx->dm.dlo, ctx->stream) ||
         launch_lowbounds(ctx->p.N, ctx->dm, kp.gamma, ctx->U, ctx->dm.dlo, stored_dt(ctx), ctx->dm.lsv,
                          ctx->dm.lob, ctx->stream)))
        return fail(ctx, DGIDP_E_DEVICE, "low-order bounds launch failed");
    HIPCHK(hipEventRecord(ev[0], ctx->stream));
    for (int r = 0; r < reps; ++r)
        if (launch_stage(ctx->p.N, ctx->dm, kp, ctx->U, nullptr, ctx->W1, 0.0, 1.0, stored_dt(ctx), nullptr,
                         ctx->stream) ||
            launch_stage(ctx->p.N, ctx->dm, kp, ctx->W1, ctx->U, ctx->W2, 0.75, 0.25, stored_dt(ctx), nullptr,
                         ctx->stream, true) ||
            launch_stage(ctx->p.N, ctx->dm, kp, ctx->W2, ctx->U, ctx->W1, 1.0 / 3.0, 2.0 / 3.0, stored_dt(ctx),
                         nullptr, ctx->stream))
            return fail(ctx, DGIDP_E_DEVICE, "stage kernel launch failed");
    HIPCHK(hipEventRecord(ev[1], ctx->stream));
    HIPCHK(hipEventRecord(ev[2], ctx->stream));
    for (int r = 0; r < reps; ++r)
        if (launch_mortar(ctx->p.N, ctx->dm, ctx->W2, 0.25, nullptr, ctx->stream, kp.gamma, kp.limiter))
            return fail(ctx, DGIDP_E_DEVICE, "mortar kernel launch failed");
    HIPCHK(hipEventRecord(ev[3], ctx->stream));
    HIPCHK(hipEventRecord(ev[4], ctx->stream));
    DtSource src;
    for (int r = 0; r < reps; ++r)
        if ((rc = enqueue_dt(ctx, 0.5, ctx->p.dt_mode, &src))) return rc;
    HIPCHK(hipEventRecord(ev[5], ctx->stream));
    HIPCHK(hipEventSynchronize(ev[5]));
    for (int k = 0; k < 3; ++k) {
        float t = 0.f;
        HIPCHK(hipEventElapsedTime(&t, ev[2 * k], ev[2 * k + 1]));
        ms[k] = (double)t / (k == 0 ? 3 * reps : reps);
    }
    for (auto& e : ev) (void)hipEventDestroy(e);
    return 0;
}

int dgidp_mesh_download(dgidp_ctx* ctx, int8_t* level, int32_t* ix, int32_t* iy)
{
    if (!ctx || !level || !ix || !iy) return DGIDP_E_INVALID_ARG;
    if (!ctx->E) return fail(ctx, DGIDP_E_NO_MESH, "no mesh");
    std::copy(ctx->level.begin(), ctx->level.end(), level);
    std::copy(ctx->ix.begin(), ctx->ix.end(), ix);
    std::copy(ctx->iy.begin(), ctx->iy.end(), iy);
    return 0;
}

int dgidp_refine_coarsen(dgidp_ctx* ctx, const int8_t* flags, double zs_eps, int64_t* n_leaves_out,
                         dgidp_adapt_stats* st)
{
    if (!ctx || !flags || !(zs_eps >= 0.0)) return DGIDP_E_INVALID_ARG;
    if (!ctx->has_state) return fail(ctx, DGIDP_E_NO_STATE, "no state");
    const int N = ctx->p.N, NN = (N + 1) * (N + 1);
    AdaptPlan plan;
    std::string err;
    int rc = adapt_leaves(ctx->E, ctx->level.data(), ctx->ix.data(), ctx->iy.data(), ctx->nx0,
                          ctx->ny0, flags, plan, err);
    if (rc) return fail(ctx, rc, err);
    const int64_t En = (int64_t)plan.level.size();
    // the new mesh must fit the index range of the kernels (the limit that
    // dgidp_mesh_upload enforces) before the current mesh and state are let go
    if (En > (int64_t)(1 << 30) / (NN * 4))
        return fail(ctx, DGIDP_E_INVALID_ARG,
                    "adaptation would give " + std::to_string(En) + " leaves, above the limit of " +
                        std::to_string((1 << 30) / (NN * 4)) + "; mesh and state kept");
    // old external -> old internal
    std::vector<int> inv_old((size_t)ctx->E);
    for (int64_t i = 0; i < ctx->E; ++i) inv_old[ctx->perm[i]] = (int)i;
    // keep the old state in its slot; the new mesh takes the other state slot
    double* uold = ctx->U;
    ctx->u_slot ^= 1;
    const double x0 = ctx->x0, y0 = ctx->y0, Lx = ctx->Lx, Ly = ctx->Ly;
    rc = dgidp_mesh_upload(ctx, En, plan.level.data(), plan.ix.data(), plan.iy.data(), x0, y0, Lx,
                           Ly, ctx->nx0, ctx->ny0);
    if (rc) return rc;
    // new external -> new internal
    std::vector<int> inv_new((size_t)En);
    for (int64_t i = 0; i < En; ++i) inv_new[ctx->perm[i]] = (int)i;
    std::vector<int> tkind((size_t)En), tsrc((size_t)En * 4, -1), zgrp;
    for (int64_t i = 0; i < En; ++i) {
        const int64_t x = ctx->perm[i];  // external id of new internal element i
        const int k = plan.kind[x];
        tkind[i] = k;
        const int64_t* sx = &plan.src[4 * x];
        if (k == 0) {
            tsrc[4 * i] = inv_old[sx[0]];
        } else if (k == 1) {
            tsrc[4 * i] = inv_old[sx[0]];
            tsrc[4 * i + 1] = (int)sx[1];
        } else {
            for (int c = 0; c < 4; ++c) tsrc[4 * i + c] = inv_old[sx[c]];
        }
    }
    for (int64_t x = 0; x < En; ++x) {
        if (plan.kind[x] == 1 && plan.src[4 * x + 1] == 0) {
            // the four children of one parent are consecutive in the new order
            zgrp.insert(zgrp.end(), {1, inv_old[plan.src[4 * x]], inv_new[x], inv_new[x + 1],
                                     inv_new[x + 2], inv_new[x + 3]});
        } else if (plan.kind[x] == 2) {
            zgrp.insert(zgrp.end(), {2, -1, inv_new[x], -1, -1, -1});
        }
    }
    const int G = (int)(zgrp.size() / 6);
    int *dk = nullptr, *ds = nullptr, *dg = nullptr;
    unsigned long long* dcount = nullptr;
    unsigned long long counts[2] = {0, 0};
    // (the transfer buffers are pool slots: nothing to free)
    auto cleanup = [&]() { (void)hipStreamSynchronize(ctx->stream); };
    if (pool_get(ctx, P_TKIND, tkind.size() * sizeof(int), dk) ||
        pool_get(ctx, P_TSRC, tsrc.size() * sizeof(int), ds) ||
        pool_get(ctx, P_TGRP, zgrp.size() * sizeof(int), dg) ||
        pool_get(ctx, P_TCOUNT, 2 * sizeof(unsigned long long), dcount) ||
        hipMemcpyAsync(dk, tkind.data(), tkind.size() * sizeof(int), hipMemcpyHostToDevice, ctx->stream) != hipSuccess ||
        hipMemcpyAsync(ds, tsrc.data(), tsrc.size() * sizeof(int), hipMemcpyHostToDevice, ctx->stream) != hipSuccess ||
        (G > 0 && hipMemcpyAsync(dg, zgrp.data(), zgrp.size() * sizeof(int), hipMemcpyHostToDevice,
                                 ctx->stream) != hipSuccess) ||
        hipMemsetAsync(dcount, 0, 2 * sizeof(unsigned long long), ctx->stream) != hipSuccess) {
        cleanup();
        return fail(ctx, DGIDP_E_DEVICE, "transfer buffers");
    }
    if (launch_transfer(N, (int)En, dk, ds, uold, ctx->U, ctx->stream) ||
        (zs_eps > 0.0 && launch_zhang_shu(N, G, dg, uold, ctx->U, zs_eps, ctx->p.gamma, dcount, ctx->stream))) {
        cleanup();
        return fail(ctx, DGIDP_E_DEVICE, "transfer kernel launch failed");
    }
    const hipError_t e1 = hipMemcpyAsync(counts, dcount, sizeof(counts), hipMemcpyDeviceToHost, ctx->stream);
    cleanup();
    if (e1 != hipSuccess) return fail(ctx, DGIDP_E_DEVICE, "transfer counters");
    ctx->has_state = true;
    if (n_leaves_out) *n_leaves_out = En;
    if (st) {
        st->n_refined = plan.n_refined;
        st->n_balance_refined = plan.n_balance;
        st->n_coarsened = plan.n_coarsened;
        st->zs_limited = (int64_t)counts[0];
        st->zs_unfixable = (int64_t)counts[1];
    }
    return 0;
}

static float* ind_staging(dgidp_ctx* ctx, size_t floats)
{
    if (ctx->ind_cap < floats) {
        dfree(ctx->ind_buf);
        ctx->ind_cap = 0;
        if (hipMalloc((void**)&ctx->ind_buf, floats * sizeof(float)) != hipSuccess) return nullptr;
        ctx->ind_cap = floats;
    }
    return ctx->ind_buf;
}

static MlpState* get_mlp(dgidp_ctx* ctx)
{
    if (!ctx->mlp) ctx->mlp = mlp_create();
    return ctx->mlp;
}

int dgidp_features(dgidp_ctx* ctx, float* f, int on_device)
{
    if (!ctx || !f) return DGIDP_E_INVALID_ARG;
    if (!ctx->has_state) return fail(ctx, DGIDP_E_NO_STATE, "no state");
    float* out = on_device ? f : ind_staging(ctx, (size_t)ctx->E * 16);
    if (!out) return fail(ctx, DGIDP_E_DEVICE, "staging buffer");
    if (launch_indicator(ctx->p.N, (int)ctx->E, ctx->U, ctx->dm.perm, ctx->p.gamma, nullptr, out,
                         ctx->stream))
        return fail(ctx, DGIDP_E_DEVICE, "indicator kernel launch failed");
    if (!on_device) {
        HIPCHK(hipMemcpyAsync(f, out, (size_t)ctx->E * 16 * sizeof(float), hipMemcpyDeviceToHost, ctx->stream));
        HIPCHK(hipStreamSynchronize(ctx->stream));
    }
    return 0;
}

int dgidp_indicator(dgidp_ctx* ctx, int kind, float* alpha, int on_device)
{
    if (!ctx || !alpha || (kind != DGIDP_IND_HENNEMANN && kind != DGIDP_IND_MLP)) return DGIDP_E_INVALID_ARG;
    if (!ctx->has_state) return fail(ctx, DGIDP_E_NO_STATE, "no state");
    const size_t E = (size_t)ctx->E;
    float* out = alpha;
    if (kind == DGIDP_IND_HENNEMANN) {
        if (!on_device && !(out = ind_staging(ctx, E))) return fail(ctx, DGIDP_E_DEVICE, "staging buffer");
        if (launch_indicator(ctx->p.N, (int)E, ctx->U, ctx->dm.perm, ctx->p.gamma, out, nullptr, ctx->stream))
            return fail(ctx, DGIDP_E_DEVICE, "indicator kernel launch failed");
    } else {
        MlpState* m = get_mlp(ctx);
        if (!m) return fail(ctx, DGIDP_E_DEVICE, "network buffers");
        if (!mlp_has_weights(m)) return fail(ctx, DGIDP_E_INVALID_ARG, "network weights not set");
        if (!on_device && !(out = ind_staging(ctx, E))) return fail(ctx, DGIDP_E_DEVICE, "staging buffer");
        if (launch_learned_indicator(ctx->p.N, (int)E, ctx->U, ctx->dm.perm, ctx->p.gamma, mlp_weights_bf16(m), out,
                                     ctx->stream))
            return fail(ctx, DGIDP_E_DEVICE, "indicator kernel launch failed");
    }
    if (!on_device) {
        HIPCHK(hipMemcpyAsync(alpha, out, E * sizeof(float), hipMemcpyDeviceToHost, ctx->stream));
        HIPCHK(hipStreamSynchronize(ctx->stream));
    }
    return 0;
}

int dgidp_mlp_set_weights(dgidp_ctx* ctx, const float* w)
{
    if (!ctx || !w) return DGIDP_E_INVALID_ARG;
    for (int i = 0; i < mlp_num_params(); ++i)
        if (!std::isfinite(w[i])) return fail(ctx, DGIDP_E_INVALID_ARG, "non-finite weight");
    MlpState* m = get_mlp(ctx);
    if (!m || mlp_set_weights(m, w, ctx->stream)) return fail(ctx, DGIDP_E_DEVICE, "network weights");
    return 0;
}

int dgidp_mlp_get_weights(dgidp_ctx* ctx, float* w)
{
    if (!ctx || !w) return DGIDP_E_INVALID_ARG;
    MlpState* m = get_mlp(ctx);
    if (!m) return fail(ctx, DGIDP_E_DEVICE, "network buffers");
    if (!mlp_has_weights(m)) return fail(ctx, DGIDP_E_INVALID_ARG, "network weights not set");
    if (mlp_get_weights(m, w, ctx->stream)) return fail(ctx, DGIDP_E_DEVICE, "network weights");
    return 0;
}

int dgidp_mlp_forward(dgidp_ctx* ctx, const float* x, int64_t B, float* y, int on_device)
{
    if (!ctx || !x || !y || B < 0 || B > (int64_t)1 << 30) return DGIDP_E_INVALID_ARG;
    MlpState* m = get_mlp(ctx);
    if (!m) return fail(ctx, DGIDP_E_DEVICE, "network buffers");
    if (!mlp_has_weights(m)) return fail(ctx, DGIDP_E_INVALID_ARG, "network weights not set");
    if (B == 0) return 0;
    if (on_device && (reinterpret_cast<uintptr_t>(x) & 15))
        return fail(ctx, DGIDP_E_INVALID_ARG, "device inputs not 16-byte aligned");
    const float* dx = x;
    float* dy = y;
    if (!on_device) {
        float* sx = mlp_scratch(m, 0, (size_t)B * 16);
        float* sy = mlp_scratch(m, 2, (size_t)B);
        if (!sx || !sy) return fail(ctx, DGIDP_E_DEVICE, "network scratch");
        HIPCHK(hipMemcpyAsync(sx, x, (size_t)B * 16 * sizeof(float), hipMemcpyHostToDevice, ctx->stream));
        dx = sx;
        dy = sy;
    }
    if (mlp_forward(m, dx, B, dy, ctx->stream)) return fail(ctx, DGIDP_E_DEVICE, "network kernel launch failed");
    if (!on_device) {
        HIPCHK(hipMemcpyAsync(y, dy, (size_t)B * sizeof(float), hipMemcpyDeviceToHost, ctx->stream));
        HIPCHK(hipStreamSynchronize(ctx->stream));
    }
    return 0;
}

static int mlp_grad_common(dgidp_ctx* ctx, const float* x, const float* t, int64_t B, float lr,
                           float* grad, float* loss, int on_device)
{
    if (!ctx || !x || !t || B <= 0 || B > (int64_t)1 << 30 || !(lr >= 0.0f)) return DGIDP_E_INVALID_ARG;
    MlpState* m = get_mlp(ctx);
    if (!m) return fail(ctx, DGIDP_E_DEVICE, "network buffers");
    if (!mlp_has_weights(m)) return fail(ctx, DGIDP_E_INVALID_ARG, "network weights not set");
    const float *dx = x, *dt = t;
    float* dg = grad;
    const size_t np = (size_t)mlp_num_params();
    if (!on_device) {
        float* sx = mlp_scratch(m, 0, (size_t)B * 16);
        float* st = mlp_scratch(m, 1, (size_t)B);
        float* sg = mlp_scratch(m, 3, np);
        if (!sx || !st || !sg) return fail(ctx, DGIDP_E_DEVICE, "network scratch");
        HIPCHK(hipMemcpyAsync(sx, x, (size_t)B * 16 * sizeof(float), hipMemcpyHostToDevice, ctx->stream));
        HIPCHK(hipMemcpyAsync(st, t, (size_t)B * sizeof(float), hipMemcpyHostToDevice, ctx->stream));
        dx = sx;
        dt = st;
        dg = grad ? sg : nullptr;
    }
    if (mlp_grad_step(m, dx, dt, B, lr, dg, loss, ctx->stream))
        return fail(ctx, DGIDP_E_DEVICE, "network kernel launch failed");
    if (!on_device && grad) {
        HIPCHK(hipMemcpyAsync(grad, dg, np * sizeof(float), hipMemcpyDeviceToHost, ctx->stream));
        HIPCHK(hipStreamSynchronize(ctx->stream));
    }
    return 0;
}

int dgidp_mlp_grad(dgidp_ctx* ctx, const float* x, const float* t, int64_t B, float* grad, float* loss,
                   int on_device)
{
    if (!grad) return DGIDP_E_INVALID_ARG;
    return mlp_grad_common(ctx, x, t, B, 0.0f, grad, loss, on_device);
}

int dgidp_mlp_train_step(dgidp_ctx* ctx, const float* x, const float* t, int64_t B, float lr,
                         float* loss, int on_device)
{
    if (!(lr > 0.0f)) return DGIDP_E_INVALID_ARG;
    return mlp_grad_common(ctx, x, t, B, lr, nullptr, loss, on_device);
}

// host copy of the operator tables (flat layout, see host_tables)
int dgidp_host_tables(int N, double* out) { return host_tables(N, out); }

}  // extern "C"
