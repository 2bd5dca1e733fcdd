// Host side of mesh adaptation (Sec. 2.4 of the paper: refinement and
// coarsening between time steps): the new leaf list from refine / coarsen
// flags with 2:1 face balance, and the three-level indicator controller.
//
// Rules (documented in include/dgidp.h, dgidp_adapt_leaves):
//  1. flag > 0 refines a leaf;
//  2. balance closure: a leaf two levels coarser than a refined neighbour's
//     children is refined as well (worklist until empty);
//  3. four sibling leaves, all flagged < 0 and none refined, become their
//     parent when no leaf touching the parent across a face has a level (after
//     rules 1-2) above parent level + 1;
//  4. new order: old order, refined leaves replaced by their children in
//     (x, y) half order (0,0) (1,0) (0,1) (1,1), coarsened groups by the
//     parent at the place of their first member.
#include <algorithm>
#include <cstdint>
#include <string>
#include <unordered_map>
#include <vector>

#include "dgidp_internal.h"
#include "dgidp_leaves.h"
#include "dgidp_par.h"

namespace dgidp {

namespace {

// a mod m in [0, m); neighbour indices are at most one period off, which
// needs no division
inline int64_t pmod(int64_t a, int64_t m)
{
    if (a >= 0 && a < m) return a;
    if (a >= -m && a < 2 * m) return a < 0 ? a + m : a - m;
    return ((a % m) + m) % m;
}

// leaves across face f of leaf e (one same-level or coarser leaf, or up to two
// finer ones); returns the count
int across(const LeafLookup& L, const int8_t* lev, const int32_t* ix, const int32_t* iy, int nx0,
           int ny0, int64_t e, int f, int64_t out[2])
{
    const int l = lev[e];
    const int64_t nxl = (int64_t)nx0 << l, nyl = (int64_t)ny0 << l;
    const int dx = f == 0 ? -1 : (f == 1 ? 1 : 0), dy = f == 2 ? -1 : (f == 3 ? 1 : 0);
    const int64_t ci = pmod(ix[e] + dx, nxl), cj = pmod(iy[e] + dy, nyl);
    int64_t s = L.get(l, ci, cj);
    if (s >= 0) {
        out[0] = s;
        return 1;
    }
    if (l > 0 && (s = L.get(l - 1, ci >> 1, cj >> 1)) >= 0) {
        out[0] = s;
        return 1;
    }
    int c = 0;
    for (int k = 0; k < 2; ++k) {
        // children of cell (ci, cj) on the side facing e
        const int64_t fi = f < 2 ? 2 * ci + (dx < 0 ? 1 : 0) : 2 * ci + k;
        const int64_t fj = f < 2 ? 2 * cj + k : 2 * cj + (dy < 0 ? 1 : 0);
        if ((s = L.get(l + 1, fi, fj)) >= 0) out[c++] = s;
    }
    return c;
}

}  // namespace

int adapt_leaves(int64_t E, const int8_t* lev, const int32_t* ix, const int32_t* iy, int nx0,
                 int ny0, const int8_t* flags, AdaptPlan& plan, std::string& err)
{
    if (E <= 0 || !lev || !ix || !iy || !flags || nx0 <= 0 || ny0 <= 0) {
        err = "invalid adaptation arguments";
        return DGIDP_E_INVALID_ARG;
    }
    for (int64_t e = 0; e < E; ++e)
        if (lev[e] >= 20 && flags[e] > 0) {
            err = "refinement beyond level 20";
            return DGIDP_E_INVALID_ARG;
        }
    LeafLookup L;
    L.build(E, lev, ix, iy, nx0, ny0);
    // rules 1-2
    std::vector<char> ref((size_t)E, 0);
    std::vector<int64_t> work;
    for (int64_t e = 0; e < E; ++e)
        if (flags[e] > 0) {
            ref[e] = 1;
            work.push_back(e);
        }
    int64_t nbal = 0;
    while (!work.empty()) {
        const int64_t e = work.back();
        work.pop_back();
        for (int f = 0; f < 4; ++f) {
            int64_t nb[2];
            const int c = across(L, lev, ix, iy, nx0, ny0, e, f, nb);
            for (int k = 0; k < c; ++k) {
                const int64_t o = nb[k];
                // e's children (level lev[e] + 1) next to o: o must reach lev[e]
                if (!ref[o] && lev[o] < lev[e]) {
                    ref[o] = 1;
                    ++nbal;
                    work.push_back(o);
                }
            }
        }
    }
    // rule 3
    std::vector<int64_t> grp((size_t)E, -1);
    int64_t ncoarse = 0;
    for (int64_t e = 0; e < E; ++e) {
        if (grp[e] >= 0 || flags[e] >= 0 || ref[e] || lev[e] == 0) continue;
        const int l = lev[e];
        const int64_t pi = ix[e] >> 1, pj = iy[e] >> 1;
        int64_t sib[4];
        bool ok = true;
        for (int c = 0; c < 4 && ok; ++c) {
            sib[c] = L.get(l, 2 * pi + (c & 1), 2 * pj + (c >> 1));
            ok = sib[c] >= 0 && flags[sib[c]] < 0 && !ref[sib[c]];
        }
        for (int c = 0; c < 4 && ok; ++c) {
            const int fx = (c & 1) ? 1 : 0, fy = (c >> 1) ? 3 : 2;  // faces on the parent's boundary
            for (int f : {fx, fy}) {
                int64_t nb[2];
                const int cnt = across(L, lev, ix, iy, nx0, ny0, sib[c], f, nb);
                for (int k = 0; k < cnt; ++k)
                    if (lev[nb[k]] + ref[nb[k]] > l) ok = false;
            }
        }
        if (!ok) continue;
        const int64_t first = *std::min_element(sib, sib + 4);
        for (int c = 0; c < 4; ++c) grp[sib[c]] = first;
        ++ncoarse;
    }
    // rule 4: each old leaf's place in the new list by a prefix count (a kept
    // leaf 1, a refined one 4, a merged group 1 at its first member), then the
    // entries written in parallel
    plan = AdaptPlan();
    plan.n_balance = nbal;
    plan.n_coarsened = ncoarse;
    std::vector<int64_t> at((size_t)E + 1, 0);
    for (int64_t e = 0; e < E; ++e) {
        const int64_t c = grp[e] >= 0 ? (grp[e] == e ? 1 : 0) : (ref[e] ? 4 : 1);
        at[e + 1] = at[e] + c;
        if (grp[e] < 0 && ref[e]) ++plan.n_refined;
    }
    const int64_t En = at[E];
    plan.level.resize(En);
    plan.ix.resize(En);
    plan.iy.resize(En);
    plan.kind.resize(En);
    plan.src.resize(En * 4);
    par_for(E, [&](int64_t lo, int64_t hi) {
        for (int64_t e = lo; e < hi; ++e) {
            const int64_t o = at[e];
            if (grp[e] >= 0) {
                if (grp[e] != e) continue;
                const int l = lev[e];
                const int64_t pi = ix[e] >> 1, pj = iy[e] >> 1;
                plan.level[o] = (int8_t)(l - 1);
                plan.ix[o] = (int32_t)pi;
                plan.iy[o] = (int32_t)pj;
                plan.kind[o] = 2;
                for (int c = 0; c < 4; ++c) plan.src[o * 4 + c] = L.get(l, 2 * pi + (c & 1), 2 * pj + (c >> 1));
            } else if (ref[e]) {
                for (int c = 0; c < 4; ++c) {
                    plan.level[o + c] = (int8_t)(lev[e] + 1);
                    plan.ix[o + c] = 2 * ix[e] + (c & 1);
                    plan.iy[o + c] = 2 * iy[e] + (c >> 1);
                    plan.kind[o + c] = 1;
                    int64_t* sp = &plan.src[(o + c) * 4];
                    sp[0] = e;
                    sp[1] = c;
                    sp[2] = sp[3] = -1;
                }
            } else {
                plan.level[o] = lev[e];
                plan.ix[o] = ix[e];
                plan.iy[o] = iy[e];
                plan.kind[o] = 0;
                int64_t* sp = &plan.src[o * 4];
                sp[0] = e;
                sp[1] = sp[2] = sp[3] = -1;
            }
        }
    });
    return 0;
}

}  // namespace dgidp

extern "C" {

int dgidp_adapt_leaves(int64_t n_leaves, const int8_t* level, const int32_t* ix, const int32_t* iy,
                       int nx0, int ny0, const int8_t* flags, int64_t capacity, int8_t* new_level,
                       int32_t* new_ix, int32_t* new_iy, int8_t* kind, int64_t* src,
                       int64_t* n_new)
{
    dgidp::AdaptPlan plan;
    std::string err;
    const int rc = dgidp::adapt_leaves(n_leaves, level, ix, iy, nx0, ny0, flags, plan, err);
    if (rc) return rc;
    const int64_t n = (int64_t)plan.level.size();
    if (n_new) *n_new = n;
    if (!new_level || !new_ix || !new_iy) return 0;
    if (capacity < n) return DGIDP_E_INVALID_ARG;
    std::copy(plan.level.begin(), plan.level.end(), new_level);
    std::copy(plan.ix.begin(), plan.ix.end(), new_ix);
    std::copy(plan.iy.begin(), plan.iy.end(), new_iy);
    if (kind) std::copy(plan.kind.begin(), plan.kind.end(), kind);
    if (src) std::copy(plan.src.begin(), plan.src.end(), src);
    return 0;
}

int dgidp_amr_flags(int64_t n, const float* indicator, const int8_t* level, int base_level,
                    int med_level, float med_threshold, int max_level, float max_threshold,
                    int8_t* flags)
{
    if (n < 0 || (n > 0 && (!indicator || !level || !flags)) || base_level < 0 ||
        med_level < base_level || max_level < med_level || !(max_threshold >= med_threshold))
        return DGIDP_E_INVALID_ARG;
    for (int64_t e = 0; e < n; ++e) {
        int target = base_level;
        if (indicator[e] >= med_threshold) target = med_level;
        if (indicator[e] >= max_threshold) target = max_level;
        flags[e] = (int8_t)(level[e] < target ? 1 : (level[e] > target ? -1 : 0));
    }
    return 0;
}

}  // extern "C"
