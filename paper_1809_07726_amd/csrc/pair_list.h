// pair_list.h -- the work list of the three pair passes (plain C++, shared by
// the host code that builds it and the kernels that decode it).
//
// Replica r with n atoms is cut into T = ceil(n/64) tiles of 64 atoms, and the
// tiles into I blocks of NI consecutive tiles.  Every unordered pair {i, j} of
// the replica belongs to exactly one item:
//   ITEM_BLOCK    (IB, J): i in I block IB (NI tiles), j in tile J, pairs with
//                 i < j.  With NI = 1 the items start at J = IB + 1 (the tile's
//                 own pairs form a triangle item); with NI > 1 at J = IB * NI,
//                 and the items whose J tile lies inside the block are masked to
//                 i < j (they keep NI independent pairs per step, which issues
//                 faster than the triangle's one).
//   ITEM_TRIANGLE (A, A):  (NI = 1 only) i, j both in tile A.  Lane l meets
//                 j = (l + k + 1) mod 64 in step k; steps 0..30 reach every
//                 pair whose index distance mod 64 is not 32 exactly once, and
//                 step 31 reaches the distance-32 pairs twice, so it runs on
//                 lanes 0..31 only.
// Encoding: x = rep | (type << 30), y = (A << 16) | B (A = IB for blocks).
#pragma once

#include <stdint.h>

#include <vector>

namespace gbr {

enum : int32_t { ITEM_BLOCK = 0, ITEM_TRIANGLE = 2 };

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
            if (ni == 1) out.push_back(make_item(r, ITEM_TRIANGLE, ib, ib));
            for (int32_t j = ni == 1 ? ib + 1 : ib * ni; j < T; ++j) out.push_back(make_item(r, ITEM_BLOCK, ib, j));
        }
    }
}

}  // namespace gbr
