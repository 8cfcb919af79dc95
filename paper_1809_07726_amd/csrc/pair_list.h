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
// Encoding: x = rep | (type << 30), y = (A << 16) | B (A = IB for blocks).
#pragma once

#include <stdint.h>

#include <algorithm>
#include <cstddef>
#include <vector>

namespace gbr {

enum : int32_t { ITEM_BLOCK = 0, ITEM_DIAG = 1, ITEM_TRIANGLE = 2 };

constexpr int32_t MAX_TILES = 65535;          // per replica (16-bit tile fields)
constexpr int32_t MAX_REPLICAS = 1 << 30;     // 30-bit replica field

struct PairItem {
    int32_t x, y;
};

inline PairItem make_item(int32_t rep, int32_t type, int32_t a, int32_t b) {
    return PairItem{rep | (type << 30), (a << 16) | b};
}

// Items of every replica in order; within a replica, I block by I block.
inline void build_pair_items(const int32_t* off, int32_t n_rep, int ni, std::vector<PairItem>& out) {
    out.clear();
    for (int32_t r = 0; r < n_rep; ++r) {
        const int32_t n = off[r + 1] - off[r];
        const int32_t T = (n + 63) / 64;
        const int32_t B = (n + 64 * ni - 1) / (64 * ni);
        for (int32_t ib = 0; ib < B; ++ib) {
            int32_t j0 = ib * ni;                   // first J tile of the block items
            if (ni == 1) {
                out.push_back(make_item(r, ITEM_TRIANGLE, ib, ib));
                j0 = ib + 1;
            } else if (ni == 2) {
                out.push_back(make_item(r, ITEM_DIAG, ib, 0));
                if (2 * ib + 1 < T) out.push_back(make_item(r, ITEM_DIAG, ib, 1));
                j0 = 2 * ib + 2;
            }
            for (int32_t j = j0; j < T; ++j) out.push_back(make_item(r, ITEM_BLOCK, ib, j));
        }
    }
    // Each eighth of the list goes to one XCD, whose wavefronts take it in
    // order: within each eighth, the 64-step block items first and the 32-step
    // triangle and diagonal items last, so that the end of the pass (when the
    // CUs drain) runs the short items.
    const size_t n = out.size(), parts = 8;
    std::vector<PairItem> tmp;
    for (size_t p = 0; p < parts; ++p) {
        const size_t b = n * p / parts, e = n * (p + 1) / parts;
        tmp.clear();
        for (size_t i = b; i < e; ++i) if (((uint32_t)out[i].x >> 30) == (uint32_t)ITEM_BLOCK) tmp.push_back(out[i]);
        for (size_t i = b; i < e; ++i) if (((uint32_t)out[i].x >> 30) != (uint32_t)ITEM_BLOCK) tmp.push_back(out[i]);
        std::copy(tmp.begin(), tmp.end(), out.begin() + (ptrdiff_t)b);
    }
}

}  // namespace gbr
