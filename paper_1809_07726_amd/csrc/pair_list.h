// pair_list.h -- the work list of the three pair passes (plain C++, shared by
// the host code that builds it and the kernels that decode it).
//
// Replica r with n atoms is cut into T = ceil(n/64) tiles of 64 atoms, and the
// tiles into I blocks of NI consecutive tiles.  Every unordered pair {i, j} of
// the replica belongs to exactly one item:
//   ITEM_BLOCK    (IB, J): i in I block IB (NI tiles), j in tile J, pairs with
//                 i < j.  With NI = 1 and NI = 2 the items start at the first
//                 tile after the block (the block's own pairs form triangle or
//                 diagonal items); with NI > 2 at J = IB * NI, and the items
//                 whose J tile lies inside the block are masked to i < j.
//   ITEM_TRIANGLE (A, A):  (NI = 1 only) i, j both in tile A.  Lane l meets
//                 j = (l + k + 1) mod 64 in step k; steps 0..30 reach every
//                 pair whose index distance mod 64 is not 32 exactly once, and
//                 step 31 reaches the distance-32 pairs twice, so it runs on
//                 lanes 0..31 only.
//   ITEM_DIAG     (IB, phase):  (NI = 2 only) the pairs inside the block's
//                 tiles a = 2 IB and b = 2 IB + 1, in two 32-step items with two
//                 independent sub-tasks each (so that a wavefront still has two
//                 pairs in flight per step, as in a block item): phase 0 = the
//                 triangles of a and of b, phase 1 = the cross pairs a x b,
//                 rotation steps 0..31 and 32..63 side by side.  Phase 1 exists
//                 only if tile b does.
// The last ceil(nb / split_den) block items of each replica's nb (in the order
// below; split_den = SPLIT_DEN unless the caller sets the split level) run as
// two halves each: rotation steps 0..31 and 32..63, the j accumulators of the
// first half ending on lane (l + 32) mod 64, those of the second back on lane
// l.  The choice depends on the replica and the split level alone, so at one
// split level a replica's results do not depend on the rest of the batch.
// Encoding: x = rep | (half << 26) | (type << 30), half = 0 (whole), 1, 2;
// y = (A << 16) | B (A = IB for blocks).
#pragma once

#include <stdint.h>

#include <algorithm>
#include <cstddef>
#include <vector>

namespace gbr {

enum : int32_t { ITEM_BLOCK = 0, ITEM_DIAG = 1, ITEM_TRIANGLE = 2, ITEM_PACKED = 3 };

constexpr int32_t MAX_TILES = 65535;          // per replica (16-bit tile fields)
constexpr int32_t MAX_REPLICAS = 1 << 26;     // 26-bit replica field
constexpr int32_t SPLIT_DEN = 16;

struct PairItem {
    int32_t x, y;
};

inline PairItem make_item(int32_t rep, int32_t type, int32_t a, int32_t b, int32_t half = 0) {
    return PairItem{rep | (half << 26) | (type << 30), (a << 16) | b};
}

// Items of every replica, within a replica I block by I block; then each
// eighth of the list reordered (below).
inline void build_pair_items(const int32_t* off, int32_t n_rep, int ni, std::vector<PairItem>& out,
                             int32_t split_den = SPLIT_DEN) {
    out.clear();
    std::vector<uint32_t> rank;                 // position of each item within its replica
    std::vector<PairItem> one;
    for (int32_t r = 0; r < n_rep; ++r) {
        const int32_t n = off[r + 1] - off[r];
        const int32_t T = (n + 63) / 64;
        const int32_t B = (n + 64 * ni - 1) / (64 * ni);
        one.clear();
        for (int32_t ib = 0; ib < B; ++ib) {
            int32_t j0 = ib * ni;                   // first J tile of the block items
            if (ni == 1) {
                one.push_back(make_item(r, ITEM_TRIANGLE, ib, ib));
                j0 = ib + 1;
            } else if (ni == 2) {
                one.push_back(make_item(r, ITEM_DIAG, ib, 0));
                if (2 * ib + 1 < T) one.push_back(make_item(r, ITEM_DIAG, ib, 1));
                j0 = 2 * ib + 2;
            }
            for (int32_t j = j0; j < T; ++j) one.push_back(make_item(r, ITEM_BLOCK, ib, j));
        }
        size_t nb = 0;
        for (const PairItem& it : one) nb += ((uint32_t)it.x >> 30) == (uint32_t)ITEM_BLOCK;
        size_t split = (nb + split_den - 1) / split_den;    // block items still to split, from the end
        for (size_t k = one.size(); k-- > 0 && split > 0;) {
            if (((uint32_t)one[k].x >> 30) != (uint32_t)ITEM_BLOCK) continue;
            one[k].x |= 1 << 26;
            --split;
        }
        for (size_t k = 0; k < one.size(); ++k) {
            out.push_back(one[k]);
            rank.push_back((uint32_t)k);
            if (((one[k].x >> 26) & 3) == 1) {
                out.push_back(PairItem{(one[k].x & ~(3 << 26)) | (2 << 26), one[k].y});
                rank.push_back((uint32_t)k);
            }
        }
    }
    // Each eighth of the list goes to one XCD, whose wavefronts take it in
    // order.  Within each eighth: the 64-step block items first and the 32-step
    // items last (triangle and diagonal items, then first halves, then second
    // halves), so that the end of the pass (when the CUs drain) runs short
    // items; and within each of these groups the replicas interleaved (items
    // ordered by their position within their replica, then by replica), so
    // that wavefronts that run at the same time (consecutive items) work on
    // different replicas and their atomic flushes go to different atoms.  The
    // order changes no result: every item's arithmetic is the same wherever it
    // sits, and fixed-point sums do not depend on order.
    auto group = [&](size_t i) -> int {
        const int half = (out[i].x >> 26) & 3;
        if (half) return 1 + half;
        return ((uint32_t)out[i].x >> 30) != (uint32_t)ITEM_BLOCK ? 1 : 0;
    };
    const size_t n = out.size(), parts = 8;
    std::vector<size_t> idx;
    std::vector<PairItem> tmp;
    for (size_t p = 0; p < parts; ++p) {
        const size_t b = n * p / parts, e = n * (p + 1) / parts;
        idx.clear();
        for (size_t i = b; i < e; ++i) idx.push_back(i);
        std::stable_sort(idx.begin(), idx.end(), [&](size_t u, size_t v) {
            const int gu = group(u), gv = group(v);
            if (gu != gv) return gu < gv;
            return rank[u] < rank[v];                   // ties keep replica order
        });
        tmp.clear();
        for (size_t i : idx) tmp.push_back(out[i]);
        std::copy(tmp.begin(), tmp.end(), out.begin() + (ptrdiff_t)b);
    }
}

// Runs with pair cutoffs replace the block items whose J tile lies after
// their I block by ITEM_PACKED items (x = rep | ITEM_PACKED << 30, y = P):
// the atoms after the block that come within the cutoff of the block, packed
// 64 at a time on the device at every evaluation.  The fixed part: the items
// whose pairs lie inside one I block (in list order); the I blocks {rep, A}
// with tiles after them, each owning as many packed tiles (from p0 on) as it
// has tiles after it (cap in all); and the windows of up to PACK_WINDOW of
// those tiles that the packing scans, {block, A << 16 | first tile, block's
// p0, replica}, block b's windows being blk_win[b] .. blk_win[b + 1] - 1.
constexpr int32_t PACK_WINDOW = 64;

struct PackWindow {
    int32_t blk, a_c0, p0, rep;
};

inline void build_packed_parts(const int32_t* off, int32_t n_rep, int ni,
                               const std::vector<PairItem>& items, std::vector<PairItem>& intra,
                               std::vector<PairItem>& iblocks, std::vector<int32_t>& p0,
                               std::vector<PackWindow>& windows, std::vector<int32_t>& blk_win,
                               int64_t& cap) {
    intra.clear();
    iblocks.clear();
    p0.clear();
    windows.clear();
    blk_win.assign(1, 0);
    cap = 0;
    for (const PairItem& it : items) {
        const bool block = ((uint32_t)it.x >> 30) == (uint32_t)ITEM_BLOCK;
        const int32_t A = (int32_t)((uint32_t)it.y >> 16), B = it.y & 0xFFFF;
        if (!block || B < (A + 1) * ni) intra.push_back(it);
    }
    for (int32_t r = 0; r < n_rep; ++r) {
        const int32_t T = (off[r + 1] - off[r] + 63) / 64;
        for (int32_t a = 0; a * ni < T; ++a) {
            const int32_t t1 = std::min(T, (a + 1) * ni);
            if (t1 >= T) continue;
            const int32_t blk = (int32_t)iblocks.size();
            iblocks.push_back(PairItem{r, a});
            p0.push_back((int32_t)cap);
            for (int32_t c0 = t1; c0 < T; c0 += PACK_WINDOW)
                windows.push_back(PackWindow{blk, (a << 16) | c0, (int32_t)cap, r});
            blk_win.push_back((int32_t)windows.size());
            cap += T - t1;
        }
    }
}

}  // namespace gbr
