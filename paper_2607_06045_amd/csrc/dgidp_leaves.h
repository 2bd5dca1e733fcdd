// Leaf lookup of a quadtree forest on an nx0 x ny0 root grid (host code).
//
// get(l, i, j) returns the index of the leaf at level l covering cell (i, j) of
// the (nx0 2^l) x (ny0 2^l) grid, or -1.  When the grids of all levels up to
// the finest leaf hold at most kDenseCells cells together, the lookup is a
// dense table per level (one 32-bit entry per cell, filled once); otherwise a
// hash map.  Mesh building and adaptation make a dozen lookups per leaf, and
// on the meshes of the paper's sizes the dense tables make them plain loads.
#pragma once

#include <cstdint>
#include <unordered_map>
#include <vector>

namespace dgidp {

class LeafLookup {
  public:
    static constexpr int64_t kDenseCells = int64_t(1) << 24;

    // Indexes the leaves; returns the first leaf that repeats an earlier one
    // (same level and cell), or -1.  Levels must lie in [0, 20] and cells
    // inside their grid (the caller checks).
    int64_t build(int64_t E, const int8_t* level, const int32_t* ix, const int32_t* iy, int nx0,
                  int ny0)
    {
        nx0_ = nx0;
        ny0_ = ny0;
        lmax_ = 0;
        for (int64_t e = 0; e < E; ++e) lmax_ = level[e] > lmax_ ? level[e] : lmax_;
        int64_t cells = 0;
        for (int l = 0; l <= lmax_ && cells <= kDenseCells; ++l) cells += ((int64_t)nx0 * ny0) << (2 * l);
        dense_ = cells <= kDenseCells;
        tab_.clear();
        map_.clear();
        if (dense_) {
            tab_.resize(lmax_ + 1);
            for (int l = 0; l <= lmax_; ++l) tab_[l].assign(((size_t)nx0 * ny0) << (2 * l), -1);
        } else {
            map_.reserve((size_t)E * 2);
        }
        int64_t dup = -1;
        for (int64_t e = 0; e < E; ++e) {
            const int l = level[e];
            if (dense_) {
                int32_t& s = tab_[l][(size_t)iy[e] * ((size_t)nx0 << l) + ix[e]];
                if (s >= 0) {
                    if (dup < 0) dup = e;
                } else {
                    s = (int32_t)e;
                }
            } else if (!map_.emplace(key(l, ix[e], iy[e]), e).second && dup < 0) {
                dup = e;
            }
        }
        return dup;
    }

    // leaf at (l, i, j), i and j inside the level-l grid; -1 if none
    int64_t get(int l, int64_t i, int64_t j) const
    {
        if (l < 0 || l > lmax_) return -1;
        if (dense_) return tab_[l][(size_t)j * ((size_t)nx0_ << l) + (size_t)i];
        auto it = map_.find(key(l, i, j));
        return it == map_.end() ? -1 : it->second;
    }

    // the same with periodic wrapping of (i, j); the remainders are taken only
    // for indices outside the grid (face neighbours of boundary leaves)
    int64_t get_wrapped(int l, int64_t i, int64_t j) const
    {
        if (l < 0 || l > lmax_) return -1;
        const int64_t nx = (int64_t)nx0_ << l, ny = (int64_t)ny0_ << l;
        if (i < 0 || i >= nx) i = ((i % nx) + nx) % nx;
        if (j < 0 || j >= ny) j = ((j % ny) + ny) % ny;
        return get(l, i, j);
    }

    int max_level() const { return lmax_; }

  private:
    static uint64_t key(int l, int64_t i, int64_t j)
    {
        return ((uint64_t)(uint32_t)l << 58) | ((uint64_t)i << 29) | (uint64_t)j;
    }
    int nx0_ = 1, ny0_ = 1, lmax_ = 0;
    bool dense_ = true;
    std::vector<std::vector<int32_t>> tab_;
    std::unordered_map<uint64_t, int64_t> map_;
};

}  // namespace dgidp
