"""The pair passes' work list (csrc/pair_list.h) built by the library's own
host code, compiled here with g++: with the kernels' masking rules (i < j in
block items, the half last step of a triangle), every unordered pair of every
replica is met exactly once, for every register blocking and for ragged
replica sizes, with the last block items of each replica split into two
halves (rotation steps 0..31 and 32..63); and the list order within each
eighth (block items first, replicas interleaved) is the one the builder
states."""
import os
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1809_07726_amd", "csrc")
# the harnesses run under AddressSanitizer and UndefinedBehaviorSanitizer
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]

HARNESS = r"""
#include <cstdio>
#include <cstdlib>
#include "pair_list.h"
int main(int argc, char** argv) {
    const int ni = std::atoi(argv[1]);                  // negative: split level 1 (every block item halved)
    std::vector<int32_t> off{0};
    for (int k = 2; k < argc; ++k) off.push_back(off.back() + std::atoi(argv[k]));
    std::vector<gbr::PairItem> items;
    gbr::build_pair_items(off.data(), (int32_t)off.size() - 1, ni < 0 ? -ni : ni, items,
                          ni < 0 ? 1 : gbr::SPLIT_DEN);
    for (const auto& it : items)
        std::printf("%d %d %d %d %d\n", it.x & 0x3FFFFFF, (int)((unsigned)it.x >> 30), it.y >> 16,
                    it.y & 0xFFFF, (it.x >> 26) & 3);
    return 0;
}
"""


@pytest.fixture(scope="module")
def harness(tmp_path_factory):
    d = tmp_path_factory.mktemp("pairlist")
    src, exe = d / "h.cpp", d / "h"
    src.write_text(HARNESS)
    subprocess.check_call(["g++", "-std=c++17", *SAN, "-I", CSRC, str(src), "-o", str(exe)])
    return str(exe)


def _items(exe, ni, sizes, split_den=16):
    """Rows (replica, type, A, B, half)."""
    out = subprocess.check_output([exe, str(ni if split_den == 16 else -ni)] + [str(s) for s in sizes], text=True)
    return np.array([list(map(int, l.split())) for l in out.splitlines()], dtype=np.int64).reshape(-1, 5)


SPLIT_DEN = 16      # the last ceil(nb / 16) block items of a replica run as halves


def _natural_items(ni, n, split_den=SPLIT_DEN):
    """(type, A, B, half) of one replica's items in their order within the
    replica: I block by I block, its triangle or diagonal items, then its block
    items; the last ceil(nb / split_den) block items as two halves each."""
    T, B = (n + 63) // 64, (n + 64 * ni - 1) // (64 * ni)
    out = []
    for ib in range(B):
        j0 = ib * ni
        if ni == 1:
            out.append((2, ib, ib))
            j0 = ib + 1
        elif ni == 2:
            out.append((1, ib, 0))
            if 2 * ib + 1 < T:
                out.append((1, ib, 1))
            j0 = 2 * ib + 2
        out += [(0, ib, j) for j in range(j0, T)]
    blocks = [k for k, it in enumerate(out) if it[0] == 0]
    split = set(blocks[len(blocks) - (len(blocks) + split_den - 1) // split_den:])
    res = []
    for k, it in enumerate(out):
        res += [(*it, 1), (*it, 2)] if k in split else [(*it, 0)]
    return res


def _rotation(lane, k):
    return (lane + k + 1) & 63


def _pairs_of_item(n, ni, typ, A, B, half):
    """Pairs (i, j) the kernels evaluate for one item, following their masks
    and step ranges."""
    lane = np.arange(64)
    out = []
    if typ == 0:                     # block: i in block A (inside the replica) x tile B, i < j
        nj = min(64, n - 64 * B)
        k0, k1 = {0: (0, 64), 1: (0, 32), 2: (32, 64)}[half]
        for k in range(k0, k1):
            m = _rotation(lane, k)
            for u in range(ni):
                i = 64 * ni * A + 64 * u + lane
                ok = (m < nj) & (i < 64 * B + m) & (i < n)
                out.append(np.stack([i[ok], 64 * B + m[ok]], -1))
        return np.concatenate(out)
    assert half == 0
    if typ == 2:                     # triangle (NI = 1): 32 rotation steps
        assert A == B and ni == 1
        nj = min(64, n - 64 * A)
        for k in range(32):
            m = _rotation(lane, k)
            ok = (m < nj) & (lane < nj) & ((k < 31) | (lane < 32))
            out.append(np.stack([64 * A + lane[ok], 64 * A + m[ok]], -1))
        return np.concatenate(out)
    assert typ == 1 and ni == 2      # diagonal item of tiles a = 2A, b = 2A + 1
    a, phase = 2 * A, B
    na, nb = min(64, n - 64 * a), min(64, n - 64 * (a + 1))
    o1 = 32 if phase else 0
    for k in range(32):
        m0, m1 = _rotation(lane, k), _rotation(lane, k + o1)
        own = (k < 31) | (lane < 32)
        if phase == 0:               # triangles of a (sub-task 0) and b (sub-task 1)
            ok0 = (m0 < na) & (lane < na) & own
            out.append(np.stack([64 * a + lane[ok0], 64 * a + m0[ok0]], -1))
            if nb > 0:
                ok1 = (m1 < nb) & (lane < nb) & own
                out.append(np.stack([64 * (a + 1) + lane[ok1], 64 * (a + 1) + m1[ok1]], -1))
        else:                        # cross pairs a x b, steps k and k + 32
            assert nb > 0
            for m in (m0, m1):
                ok = m < nb
                out.append(np.stack([64 * a + lane[ok], 64 * (a + 1) + m[ok]], -1))
    return np.concatenate(out)


@pytest.mark.parametrize("split_den", [16, 1])
@pytest.mark.parametrize("ni", [1, 2, 4, 8])
def test_every_pair_exactly_once(harness, ni, split_den):
    """At the default split level and with every block item halved."""
    sizes = [1, 2, 63, 64, 65, 127, 128, 129, 200, 511, 640, 1000, 3000]
    items = _items(harness, ni, sizes, split_den)
    # each eighth of the list (one XCD's share): 64-step block items first, then
    # the 32-step triangle and diagonal items; within each group the replicas
    # interleaved: items by their position within their replica, then replica
    N = len(items)
    natural = [_natural_items(ni, n, split_den) for n in sizes]
    assert sorted(map(tuple, items.tolist())) == sorted(
        (r, *it) for r, its in enumerate(natural) for it in its)
    # rank: position of the (whole) item within its replica, halves sharing it
    whole = [[it[:3] for k, it in enumerate(nat) if it[3] != 2] for nat in natural]
    rank = np.array([whole[r].index((t, a, b)) for r, t, a, b, h in items.tolist()])
    group = np.where(items[:, 4] > 0, 1 + items[:, 4], (items[:, 1] != 0).astype(np.int64))
    for p in range(8):
        sl = slice(N * p // 8, N * (p + 1) // 8)
        key = group[sl] * 10**9 + rank[sl] * 10**3 + items[sl, 0]
        assert np.all(np.diff(key) > 0), p
    for r, n in enumerate(sizes):
        its = items[items[:, 0] == r]
        P = np.concatenate([_pairs_of_item(n, ni, *it[1:]) for it in its]) if len(its) else np.zeros((0, 2), int)
        assert np.all(P[:, 0] != P[:, 1]), (n, ni)
        assert P.min(initial=0) >= 0 and P.max(initial=0) < n
        a, b = np.minimum(P[:, 0], P[:, 1]), np.maximum(P[:, 0], P[:, 1])
        key = a * n + b
        assert key.size == n * (n - 1) // 2, (n, ni, key.size)
        assert np.unique(key).size == key.size, (n, ni)


def test_item_counts_per_replica(harness):
    """NI = 1: one triangle per tile and one block item per later tile; NI = 2:
    two diagonal items per two-tile block and one block item per later tile;
    NI > 2: one block item per tile from the block's first tile on."""
    def blocks(items):              # block items, a split one counted once
        return ((items[:, 1] == 0) & (items[:, 4] != 2)).sum()

    items = _items(harness, 1, [1024])
    assert (items[:, 1] == 2).sum() == 16 and blocks(items) == 16 * 15 // 2
    assert (items[:, 4] == 1).sum() == (items[:, 4] == 2).sum() == 8        # ceil(120 / 16)
    items = _items(harness, 2, [1024])
    assert (items[:, 1] == 1).sum() == 16 and blocks(items) == sum(16 - 2 * ib - 2 for ib in range(8))
    assert (items[:, 4] == 1).sum() == 4                                    # ceil(56 / 16)
    items = _items(harness, 2, [64 * 15])           # last block has one tile: no cross phase
    assert (items[:, 1] == 1).sum() == 15
    items = _items(harness, 4, [1024])
    assert (items[:, 1] == 0).all() and blocks(items) == sum(16 - 4 * ib for ib in range(4))
    assert (items[:, 4] == 1).sum() == 3                                    # ceil(40 / 16)


@pytest.mark.parametrize("K,o", [(32, 0), (64, 0), (32, 32)])
def test_rotating_accumulator_lands_on_lane_plus_k(K, o):
    """acc <- acc[lane + 1] + c with c the contribution of lane l to
    j = (l + k + o + 1) mod 64 (o: the first rotation step, 32 for a diagonal
    item's second sub-task and for the second half of a block item): after K
    steps lane l holds the sum for j = (l + K + o) mod 64, which is where the
    kernels flush it."""
    rng = np.random.default_rng(K + o)
    lane = np.arange(64)
    contrib = np.zeros(64)
    acc = np.zeros(64)
    for k in range(K):
        c = rng.normal(size=64)
        j = (lane + k + o + 1) & 63
        np.add.at(contrib, j, c)
        acc = np.roll(acc, -1) + c
    assert np.allclose(acc, contrib[(lane + K + o) & 63], rtol=0, atol=1e-12)


PACK_HARNESS = r"""
#include <cstdio>
#include <cstdlib>
#include "pair_list.h"
int main(int argc, char** argv) {
    const int ni = std::atoi(argv[1]);
    std::vector<int32_t> off{0};
    for (int k = 2; k < argc; ++k) off.push_back(off.back() + std::atoi(argv[k]));
    std::vector<gbr::PairItem> items, intra, blocks;
    std::vector<int32_t> p0;
    std::vector<gbr::PackWindow> wins;
    std::vector<int32_t> blk_win;
    int64_t cap = 0;
    gbr::build_pair_items(off.data(), (int32_t)off.size() - 1, ni, items);
    gbr::build_packed_parts(off.data(), (int32_t)off.size() - 1, ni, items, intra, blocks, p0, wins, blk_win,
                            cap);
    std::printf("cap %lld\n", (long long)cap);
    for (const auto& it : intra)
        std::printf("I %d %d %d %d %d\n", it.x & 0x3FFFFFF, (int)((unsigned)it.x >> 30), it.y >> 16,
                    it.y & 0xFFFF, (it.x >> 26) & 3);
    for (size_t b = 0; b < blocks.size(); ++b)
        std::printf("B %d %d %d %d %d\n", blocks[b].x, blocks[b].y, p0[b], blk_win[b], blk_win[b + 1]);
    for (const auto& w : wins) std::printf("W %d %d %d %d %d\n", w.blk, w.a_c0 & 0xFFFF, w.p0, w.a_c0 >> 16, w.rep);
    return 0;
}
"""


@pytest.fixture(scope="module")
def pack_harness(tmp_path_factory):
    d = tmp_path_factory.mktemp("packparts")
    src, exe = d / "p.cpp", d / "p"
    src.write_text(PACK_HARNESS)
    subprocess.check_call(["g++", "-std=c++17", *SAN, "-I", CSRC, str(src), "-o", str(exe)])
    return str(exe)


@pytest.mark.parametrize("ni", [1, 2, 4, 8])
def test_packed_lists_cover_every_pair_once(harness, pack_harness, ni):
    """With pair cutoffs the passes run the intra-block items plus, for every
    I block with tiles after it, packed items holding (at most) every atom
    after the block.  With a radius that keeps every atom, the intra-block
    items and the block-times-later-atoms pairs meet every pair of every
    replica exactly once; each block owns one packed tile per tile after it
    (enough for all those atoms), its windows cover those tiles once in
    pieces of at most 64, and the intra items keep the list's order."""
    sizes = [1, 63, 64, 65, 200, 511, 640, 1000, 2100]
    out = subprocess.check_output([pack_harness, str(ni)] + [str(s) for s in sizes], text=True).splitlines()
    cap = int(out[0].split()[1])
    intra = np.array([list(map(int, l.split()[1:])) for l in out if l[0] == "I"], np.int64).reshape(-1, 5)
    blocks = np.array([list(map(int, l.split()[1:])) for l in out if l[0] == "B"], np.int64).reshape(-1, 5)
    wins = np.array([list(map(int, l.split()[1:])) for l in out if l[0] == "W"], np.int64).reshape(-1, 5)
    full = _items(harness, ni, sizes)
    A_, B_ = full[:, 2], full[:, 3]
    inside = (full[:, 1] != 0) | (B_ < (A_ + 1) * ni)
    assert np.array_equal(intra, full[inside])
    p_next = 0
    for b, (r, A, p0, wb, we) in enumerate(blocks):
        n = sizes[r]
        T = (n + 63) // 64
        t1 = min(T, (A + 1) * ni)
        assert t1 < T and p0 == p_next
        p_next += T - t1
        w = wins[wins[:, 0] == b]
        assert np.array_equal(np.flatnonzero(wins[:, 0] == b), np.arange(wb, we))   # the block's window range
        tiles = np.concatenate([np.arange(c0, min(c0 + 64, T)) for c0 in w[:, 1]])
        assert np.array_equal(tiles, np.arange(t1, T)) and np.all(w[:, 2] == p0)
        assert np.all(w[:, 3] == A) and np.all(w[:, 4] == r)
    assert cap == p_next
    for r, n in enumerate(sizes):
        its = intra[intra[:, 0] == r]
        P = [_pairs_of_item(n, ni, *it[1:]) for it in its]
        for (rr, A, p0, _, _) in blocks[blocks[:, 0] == r]:
            T = (n + 63) // 64
            t1 = min(T, (A + 1) * ni)
            i = np.arange(64 * ni * A, 64 * t1)
            j = np.arange(64 * t1, n)
            P.append(np.stack(np.meshgrid(i, j, indexing="ij"), -1).reshape(-1, 2))
        P = np.concatenate(P) if P else np.zeros((0, 2), int)
        a, bb = np.minimum(P[:, 0], P[:, 1]), np.maximum(P[:, 0], P[:, 1])
        assert np.all(a != bb) and P.max(initial=0) < n
        key = a * n + bb
        assert key.size == n * (n - 1) // 2 and np.unique(key).size == key.size, (n, ni)
