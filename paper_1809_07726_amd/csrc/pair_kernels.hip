// pair_kernels.hip -- the three O(N^2) pair passes of a GB evaluation.
//
// Work decomposition (same for the three passes; the item list is described
// in pair_list.h).  One wavefront processes one item.  In a block item lane l
// holds the NI atoms i = IB*64*NI + u*64 + l (u < NI) in registers; in a
// square or triangle item it holds one atom of tile A.  The j tile is copied
// to a per-wavefront LDS slice.
//
// Rotating j accumulators: in step k lane l pairs its i atoms with
// j = (l + k + 1) mod 64, read from LDS, and adds its contribution into a
// per-lane accumulator that is first rotated by one lane (DPP wave_rol:1,
// folded into the add).  The accumulator that lane l adds into in step k
// therefore always belongs to the j it is working on; an item that runs steps
// k0 .. k1 - 1 (0 .. 63 for a block, 0 .. 31 or 32 .. 63 for half of one, 0 ..
// 31 for a triangle) ends with lane l holding the accumulator of
// j = (l + k1) mod 64.  This replaces a 64-lane reduction per j with one DPP
// add per component per step.
//
// Contributions to i accumulate per lane in FP32.  At the end of the item
// every per-atom partial is rounded to 64-bit fixed point and added with an
// integer atomic, so the result does not depend on the order in which items
// run.  Invalid pairs (j past the end of the replica, i lanes past the end of
// a ragged triangle, the duplicated half of a triangle's last step) are
// removed by zeroing 1/r (or sending r to 1e15 A), which makes every term of
// the pair exactly zero; items on full tiles run an unmasked loop.
//
// Items are visited grid-stride by a persistent grid whose block index is
// remapped so that the blocks of one XCD (blocks are dealt round-robin to the
// eight XCDs) walk a contiguous range of the item list, i.e. of replicas.
#include <algorithm>
#include <cfloat>
#include <type_traits>

#include <hip/hip_ext.h>

#include "gbr_device.h"
#include "gbr_internal.h"
#include "pair_list.h"

using namespace gbr;

// Salt screening and pair cutoffs as the pair kernels use them (the EXT
// variants; with kappa = 0 and no cutoffs the plain variants run):
// kl2e = kappa log2(e), a = eps_in / eps_out, ak = a kappa, cut2 = cut^2 and
// rgb2 = rgbmax^2 (FLT_MAX when off).  With both cutoffs the list holds packed
// items, whose J atoms are listed in pk_j (64 per packed tile, replica-local
// indices) with pk_hdr[P] = A << 7 | nj.
struct PairExt {
    float kl2e, a, ak, cut2, rgb2;
    const int32_t* pk_hdr;
    const int32_t* pk_j;
};

namespace {

constexpr float FAR_R2 = 1.0e30f;       // r^2 used for masked pairs
constexpr float LOG2E = 1.4426950408889634f;

__device__ __forceinline__ int logical_wave() {
    const int nb = gridDim.x, b = blockIdx.x;
    const int lb = (nb & 7) ? b : ((b & 7) * (nb >> 3) + (b >> 3));
    return lb * (blockDim.x >> 6) + wave_in_group();
}

// acc <- acc[lane + 1 (mod 64)] + c : rotate-and-add, one VALU instruction.
// The rotation gives every lane a source, so the DPP "old" value is never
// used.  SELF passes acc itself as old, which lets the destination reuse
// acc's register instead of a zeroed copy; which form schedules better
// differs by kernel (measured on the loop bodies).
template <bool SELF = false>
__device__ __forceinline__ float rot_add(float acc, float c) {
    const int a = __builtin_bit_cast(int, acc);
    return c + __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(
                   SELF ? a : 0, a, 0x134 /* wave_rol:1 */, 0xF, 0xF, false));
}

__device__ __forceinline__ void wave_lds_fence() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

struct ItemGeom {
    int rep, a0, n, ibase, jbase, nj;
    int u_lim;      // i sub-blocks with a valid pair
    bool tri;       // triangle item (NI = 1 only)
    bool diag;      // diagonal item of a two-tile block (NI = 2 only)
    bool packed;    // packed item: J atoms listed in jx (PK variants only)
    int phase;      // diagonal item: 0 = both tiles' own pairs, 1 = the cross pairs
    int k0, k1;     // rotation steps k0 .. k1 - 1 of the item
    const int32_t* jx;
};

// PK: the list may hold packed items (the EXT variants).  A packed item's I
// block is always whole (atoms exist after it) and its J atoms all follow the
// block, so its only invalid pairs are the empty J slots m >= nj.
template <int NI, bool PK>
__device__ __forceinline__ ItemGeom item_geom(const int2 wi, const int32_t* __restrict__ atom_off,
                                              const PairExt& ext) {
    ItemGeom g;
    g.rep = wi.x & 0x3FFFFFF;
    const int type = (int)((unsigned)wi.x >> 30);
    const int half = (wi.x >> 26) & 3;              // block items: 0 whole, 1 / 2 halves
    const int A = (int)((unsigned)wi.y >> 16), B = wi.y & 0xFFFF;
    g.a0 = atom_off[g.rep];
    g.n = atom_off[g.rep + 1] - g.a0;
    g.tri = NI == 1 && type == ITEM_TRIANGLE;
    g.diag = NI == 2 && type == ITEM_DIAG;
    g.packed = PK && type == ITEM_PACKED;
    g.jx = nullptr;
    if (PK && g.packed) {
        const int P = wi.y;
        const int h = ext.pk_hdr[P];
        g.phase = 0;
        g.ibase = (h >> 7) * 64 * NI;
        g.jbase = 0;
        g.nj = h & 127;
        g.jx = ext.pk_j + (int64_t)P * 64;
        g.u_lim = NI;
        g.k0 = 0;
        g.k1 = 64;
    } else if (NI == 2 && g.diag) {
        g.phase = B;
        g.ibase = A * 128;                              // tile a; tile b follows it
        g.jbase = g.phase ? g.ibase + 64 : g.ibase;     // tile of LDS slot 0
        g.nj = min(64, g.n - g.jbase);
        g.u_lim = g.ibase + 64 < g.n ? 2 : 1;           // tile b exists
        g.k0 = 0;
        g.k1 = 32;
    } else {
        g.phase = 0;
        g.ibase = A * 64 * NI;
        g.jbase = B * 64;
        g.nj = min(64, g.n - g.jbase);
        g.k0 = half == 2 ? 32 : 0;
        g.k1 = (g.tri || half == 1) ? 32 : 64;
        // I sub-blocks u with a valid pair: ibase + 64u < jbase + nj (and < n)
        const int span = g.jbase + g.nj - g.ibase;
        g.u_lim = min(NI, (span + 63) >> 6);
    }
    return g;
}

// i atom of sub-block u (the cross phase of a diagonal item holds tile a in
// both sub-blocks).
template <int NI>
__device__ __forceinline__ int item_li(const ItemGeom& g, int u, int lane) {
    return (NI == 2 && g.diag && g.phase == 1) ? g.ibase + lane : g.ibase + u * 64 + lane;
}

// Validity of the pair of sub-block u in the masked loop (step k, j tile slot
// m): j inside the replica and, in a block item on the diagonal, i < j; in a
// triangle both atoms inside the replica and only lanes 0..31 on step 31.
template <int NI, bool PK>
__device__ __forceinline__ bool pair_ok(const ItemGeom& g, int lane, int k, int m, int li) {
    const bool jok = m < g.nj;
    if (PK && g.packed) return jok;
    if (NI == 1 && g.tri) return jok & (lane < g.nj) & ((k < 31) | (lane < 32));
    return jok & (li < g.jbase + m);
}

// Replica-local index of J slot m (g.n for an empty slot).
template <bool PK>
__device__ __forceinline__ int j_of_slot(const ItemGeom& g, int m) {
    if (PK && g.packed) return m < g.nj ? g.jx[m] : g.n;
    return g.jbase + m;
}

// Replica-local atom loaded into J slot `lane` of a tile starting at tb (a
// packed item's listed atom; past the end the last valid one).
template <bool PK>
__device__ __forceinline__ int j_fill(const ItemGeom& g, int tb, int lane) {
    if (PK && g.packed) return g.jx[min(lane, g.nj - 1)];
    return min(tb + lane, g.n - 1);
}

// Runs the item's steps through kloop(full, k0, k1): unmasked where every pair
// is valid (a block item entirely before a full j tile; steps 0..30 of a
// triangle on a full tile), masked for the rest.  Each variant is called from
// one place so that it is inlined.
template <int NI, bool PK, typename K>
__device__ __forceinline__ void run_item(const ItemGeom& g, K& kloop) {
    if constexpr (NI == 1) {
        int f1 = g.k0;
        if (g.nj == 64) f1 = g.tri ? 31 : g.k1;
        if (f1 > g.k0) kloop(std::true_type{}, g.k0, f1);
        if (f1 < g.k1) kloop(std::false_type{}, f1, g.k1);
    } else {
        const bool full = (PK && g.packed) ? g.nj == 64 : (g.nj == 64 && g.ibase + 64 * NI <= g.jbase);
        if (full) kloop(std::true_type{}, g.k0, g.k1);
        else kloop(std::false_type{}, g.k0, g.k1);
    }
}

// Diagonal item of a two-tile block (tiles a, b; NI = 2), two independent
// sub-tasks per step so that a wavefront keeps two pairs in flight:
//   phase 0: sub-task 0 = the pairs inside tile a, sub-task 1 = inside tile b,
//            each as a triangle (32 steps, step 31 on lanes 0..31 only), j from
//            LDS slots 0 (tile a) and 1 (tile b);
//   phase 1: the cross pairs a x b, sub-task 0 taking rotation steps 0..31 and
//            sub-task 1 steps 32..63, both with j from slot 0 (tile b).
// step(m0, m1, ok0, ok1) receives each sub-task's j slot index and validity.
// After the 32 steps sub-task u's j accumulators sit at j = (l + 32 + o_u) mod
// 64 of their tile, o_1 = 32 in phase 1 and 0 otherwise.
template <typename F>
__device__ __forceinline__ void run_diag(const ItemGeom& g, int lane, F&& step) {
    const int o1 = g.phase ? 32 : 0;
    const int na = min(64, g.n - g.ibase), nb = min(64, g.n - g.ibase - 64);
    const int nt0 = g.phase ? nb : na;
    for (int k = 0; k < 32; ++k) {
        const int m0 = (lane + k + 1) & 63, m1 = (lane + k + o1 + 1) & 63;
        const bool own = (k < 31) | (lane < 32);
        const bool ok0 = (m0 < nt0) & (g.phase | ((lane < nt0) & own));
        const bool ok1 = (m1 < nb) & (g.phase | ((lane < nb) & own));
        step(m0, m1, ok0, ok1);
    }
}

// Far-sphere test for both descreening directions of a pair: with
// m = max(rt, s) and sx = s / HCT_FAR_XMAX per atom, r >= max(m_i + m_j,
// sx_i, sx_j) implies r - s_j >= rt_i, r - s_i >= rt_j and s/r <= XMAX for both
// spheres, so both terms may use the polynomial form.
__device__ __forceinline__ bool both_far(float r, float mi, float mj, float sxi, float sxj) {
    return r >= fmaxf(mi + mj, fmaxf(sxi, sxj));
}

// Items generated from the wavefront index instead of read from a list (the
// context-free descreening pass, NI = 1): it = (rep T + A) T + B over the
// replicas and the 64-atom tiles of the largest replica (T of them); A == B is
// tile A's triangle item, B > A the block item (A, B); an index with B < A or
// a tile past the end of its replica carries no item.  A replica that does
// not fit T tiles, or that reaches past ntot atoms, sets GBR_ERR_LAYOUT and
// is skipped.
__device__ __forceinline__ bool gen_item(int it, int T, const int32_t* __restrict__ atom_off, int ntot,
                                         uint32_t* err, int2& wi) {
    const int TT = T * T;
    const int rep = it / TT, rem = it - rep * TT;
    const int A = rem / T, B = rem - A * T;
    if (B < A) return false;
    const int a0 = atom_off[rep], a1 = atom_off[rep + 1];
    if (a0 < 0 || a1 < a0 || a1 > ntot || a1 - a0 > 64 * T) {
        if (A == 0 && B == 0) raise_error(err, GBR_ERR_LAYOUT);
        return false;
    }
    if (B * 64 >= a1 - a0) return false;
    wi = make_int2(rep | ((A == B ? ITEM_TRIANGLE : ITEM_BLOCK) << 30), (A << 16) | B);
    return true;
}

// ------------------------------------------------------------- descreening
// Distant spheres: h = (x^3/r) G(x^2) with x = s/r, i.e. h = s^3 r^-4 G(s^2 r^-2).
// j tile in LDS: {x, y, z, s}, {rt, m, sx, s^3}
// GEN: items from gen_item (gen_T tiles per replica at most) instead of a list.
template <int NI, bool EXT, bool GEN = false>
__global__ __launch_bounds__(256) void k_born_pair(
    const int2* __restrict__ items, int n_items, const int32_t* __restrict__ n_dev,
    const int32_t* __restrict__ atom_off, int ntot,
    const float* __restrict__ xyz, const float* __restrict__ rho,
    const float* __restrict__ screen, float offset, PairExt ext, int64_t* __restrict__ psi_fx,
    uint32_t* __restrict__ err, int gen_T = 0)
{
    static_assert(!GEN || NI == 1, "generated items are one-tile items");
    constexpr int NSL = NI == 2 ? 2 : 1;           // j tiles per wavefront
    extern __shared__ float4 lds_dyn[];          // j tiles: [waves in the group][NSL][2][64]
    auto lds = reinterpret_cast<float4 (*)[NSL][2][64]>(lds_dyn);
    const int lane = threadIdx.x & 63, wv = wave_in_group();
    const int stride = gridDim.x * (blockDim.x >> 6);
    const float ixmax = 1.0f / HCT_FAR_XMAX;
    if (n_dev) n_items = n_dev[0];                // a packed list: its device count
    for (int it = logical_wave(); it < n_items; it += stride) {
        int2 wi;
        if constexpr (GEN) {
            if (!gen_item(it, gen_T, atom_off, ntot, err, wi)) continue;
        } else {
            wi = items[it];
        }
        const ItemGeom g = item_geom<NI, EXT>(wi, atom_off, ext);
        float xi[NI], yi[NI], zi[NI], rti[NI], si[NI], s2i[NI], s3i[NI], mi[NI], sxi[NI], acc[NI];
        int li[NI];
#pragma unroll
        for (int u = 0; u < NI; ++u) {
            li[u] = item_li<NI>(g, u, lane);
            const int a = g.a0 + min(li[u], g.n - 1);
            xi[u] = xyz[a]; yi[u] = xyz[ntot + a]; zi[u] = xyz[2 * ntot + a];
            rti[u] = rho[a] - offset;
            si[u] = screen[a] * rti[u];
            s2i[u] = si[u] * si[u];
            s3i[u] = s2i[u] * si[u];
            mi[u] = fmaxf(rti[u], si[u]);
            sxi[u] = si[u] * ixmax;
            acc[u] = 0.0f;
        }
        auto fill = [&](int slot, int tb) {
            const int ja = g.a0 + j_fill<EXT>(g, tb, lane);
            const float rt = rho[ja] - offset, s = screen[ja] * rt;
            lds[wv][slot][0][lane] = make_float4(xyz[ja], xyz[ntot + ja], xyz[2 * ntot + ja], s);
            lds[wv][slot][1][lane] = make_float4(rt, fmaxf(rt, s), s * ixmax, s * s * s);
        };
        fill(0, g.jbase);
        if (NSL > 1 && g.diag && g.phase == 0 && g.u_lim > 1) fill(NSL - 1, g.ibase + 64);
        wave_lds_fence();
        float accj[NSL];
#pragma unroll
        for (int t = 0; t < NSL; ++t) accj[t] = 0.0f;
        // sub-block u against j data (p0, p1): adds h_ij to i, returns h_ji
        auto pair = [&](int u, const float4& p0, const float4& p1, bool ok, auto full) -> float {
            constexpr bool FULL = decltype(full)::value;
            const float sj = p0.w, s2j = sj * sj;
            const float dx = p0.x - xi[u], dy = p0.y - yi[u], dz = p0.z - zi[u];
            float r2 = dx * dx + dy * dy + dz * dz;
            if (!FULL) r2 = ok ? r2 : FAR_R2;
            if (EXT) r2 = r2 < ext.rgb2 ? r2 : FAR_R2;      // descreening cutoff
            const float rinv = frsq(r2);
            const float rinv2 = rinv * rinv;
            const float rinv4 = rinv2 * rinv2;
            float hij = (p1.w * rinv4) * poly_G(s2j * rinv2);
            float hji = (s3i[u] * rinv4) * poly_G(s2i[u] * rinv2);
            const float r = r2 * rinv;
            if (!both_far(r, mi[u], p1.y, sxi[u], p1.z)) {
                hij = (r + sj <= rti[u]) ? 0.0f : hct_closed(r, rinv, rti[u], sj);
                hji = (r + si[u] <= p1.x) ? 0.0f : hct_closed(r, rinv, p1.x, si[u]);
            }
            acc[u] += hij;
            return hji;
        };
        auto kloop = [&](auto full, int k0, int k1) {
            constexpr bool FULL = decltype(full)::value;
            for (int k = k0; k < k1; ++k) {
                const int m = (lane + k + 1) & 63;
                const float4 p0 = lds[wv][0][0][m], p1 = lds[wv][0][1][m];
                float cj = 0.0f;
#pragma unroll
                for (int u = 0; u < NI; ++u) {
                    if (FULL || u < g.u_lim) {
                        const float h = pair(u, p0, p1, FULL || pair_ok<NI, EXT>(g, lane, k, m, li[u]), full);
                        cj = (u == 0) ? h : cj + h;
                    }
                }
                accj[0] = rot_add(accj[0], cj);
            }
        };
        if constexpr (NI == 2) {
            if (g.diag) {
                const int s1 = g.phase ? 0 : NSL - 1;
                run_diag(g, lane, [&](int m0, int m1, bool ok0, bool ok1) {
                    accj[0] = rot_add(accj[0], pair(0, lds[wv][0][0][m0], lds[wv][0][1][m0], ok0,
                                                    std::false_type{}));
                    if (g.u_lim > 1)
                        accj[NSL - 1] = rot_add(accj[NSL - 1], pair(1, lds[wv][s1][0][m1], lds[wv][s1][1][m1],
                                                                    ok1, std::false_type{}));
                });
            } else {
                run_item<NI, EXT>(g, kloop);
            }
        } else {
            run_item<NI, EXT>(g, kloop);
        }
        wave_lds_fence();
#pragma unroll
        for (int u = 0; u < NI; ++u)
            if (u < g.u_lim && li[u] < g.n)
                atomic_add_fx(&psi_fx[g.a0 + li[u]], to_fixed_f(acc[u], FXF_FORCE, err));
        const int jl = j_of_slot<EXT>(g, (lane + g.k1) & 63);
        if (jl < g.n) atomic_add_fx(&psi_fx[g.a0 + jl], to_fixed_f(accj[0], FXF_FORCE, err));
        if (NSL > 1 && g.diag && g.u_lim > 1) {
            const int jl1 = g.ibase + 64 + ((lane + (g.phase ? 64 : 32)) & 63);
            if (jl1 < g.n) atomic_add_fx(&psi_fx[g.a0 + jl1], to_fixed_f(accj[NSL - 1], FXF_FORCE, err));
        }
    }
}

// ---------------------------------------------- energy and direct forces
// Per-atom scaled inputs: qc = q sqrt(k_e/eps_in), L2 = sqrt(log2(e)/4)/R,
// hs = sigma/2, se = 2 sqrt(eps).  Per pair at fixed Born radii, with
// tau' = tau eps_in and D = r^2/(4 R_i R_j):
//   e_C  = qc_i qc_j / r
//   e_GB = -tau' qc_i qc_j / f,  f^2 = r^2 + R_i R_j exp(-D)
//   e_LJ = 4 eps_ij (s^12 - s^6),  s = sigma_ij / r
//   (1/r) dE/dr = -(e_C + 6 e4 (2 s^12 - s^6)) / r^2 + tau' (qc_i qc_j / f^3)(1 - exp(-D)/4)
//   dE/dR_i = tau' (qc_i qc_j / f^3) exp(-D) (1 + D) R_j / 2
//   dE/dq_i = sqrt(k_e/eps_in) (1/r - tau'/f) qc_j
// The factors tau' and sqrt(k_e/eps_in) are applied once per atom at the flush.
// j tile in LDS: {x, y, z, qc}, {R, L2, hs, se}.
struct EnergyJ {
    float x, y, z, R, q;
};

template <int NI, bool GQ, bool EXT>
__global__ __launch_bounds__(256) void k_energy_pair(
    const int2* __restrict__ items, int n_items, const int32_t* __restrict__ n_dev,
    const int32_t* __restrict__ atom_off, int ntot,
    const float* __restrict__ xyz, const float* __restrict__ q, const float* __restrict__ Rb,
    const float* __restrict__ sigma, const float* __restrict__ eps, float sq_ke_in, float taup, PairExt ext,
    int64_t* __restrict__ force_fx, int64_t* __restrict__ dEdR_fx,
    int64_t* __restrict__ e_stripe, int64_t* __restrict__ dEdq_fx, uint32_t* __restrict__ err)
{
    constexpr int NSL = NI == 2 ? 2 : 1;
    // j tiles per wavefront (energy_lds): slot 0 as [2][128], each component's
    // 64 entries stored twice so that step k reads entry lane + k + 1 without
    // wrapping; slot 1 (diagonal items' tile b) as [2][64]
    extern __shared__ float4 lds_dyn[];
    const int lane = threadIdx.x & 63, wv = wave_in_group();
    float4* const w0 = lds_dyn + wv * (256 + (NSL - 1) * 128);
    float4* const w1 = w0 + 256;
    const int stride = gridDim.x * (blockDim.x >> 6);
    const float lc = 0.60056120439322491f;       // sqrt(log2(e) / 4)
    const float hl = 0.5f / LOG2E;               // D = D2 / log2(e)
    const float wq = -0.25f * taup;
    if (n_dev) n_items = n_dev[0];                // a packed list: its device count
    // energy sums of the wavefront's current replica (valid in lane 63); one
    // set of atomics per replica change rather than per item, into the stripe
    // of the replica that this wavefront's index selects
    int e_rep = -1;
    long long e_sum[3] = {0, 0, 0};
    const int e_str = logical_wave() & (E_STRIPES - 1);
    auto flush_e = [&]() {
        if (e_rep >= 0 && lane == 63) {
            int64_t* d = e_stripe + ((size_t)e_rep * E_STRIPES + e_str) * E_STRIPE_LEN;
            atomic_add_fx(&d[0], e_sum[0]);
            atomic_add_fx(&d[1], e_sum[1]);
            atomic_add_fx(&d[2], e_sum[2]);
        }
        e_sum[0] = e_sum[1] = e_sum[2] = 0;
    };
    for (int it = logical_wave(); it < n_items; it += stride) {
        const ItemGeom g = item_geom<NI, EXT>(items[it], atom_off, ext);
        float xi[NI], yi[NI], zi[NI], qi[NI], Ri[NI], Li[NI], hsi[NI], sei[NI];
        float fxi[NI], fyi[NI], fzi[NI], dRi[NI], dqi[NI];
        int li[NI];
#pragma unroll
        for (int u = 0; u < NI; ++u) {
            li[u] = item_li<NI>(g, u, lane);
            const int a = g.a0 + min(li[u], g.n - 1);
            xi[u] = xyz[a]; yi[u] = xyz[ntot + a]; zi[u] = xyz[2 * ntot + a];
            qi[u] = q[a] * sq_ke_in;
            Ri[u] = Rb[a];
            Li[u] = lc / Ri[u];
            hsi[u] = 0.5f * sigma[a];
            sei[u] = 2.0f * sqrtf(eps[a]);
            fxi[u] = fyi[u] = fzi[u] = dRi[u] = dqi[u] = 0.0f;
        }
        auto fill = [&](int slot, int tb) {
            const int ja = g.a0 + j_fill<EXT>(g, tb, lane);
            const float Rj = Rb[ja];
            const float4 v0 = make_float4(xyz[ja], xyz[ntot + ja], xyz[2 * ntot + ja], q[ja] * sq_ke_in);
            const float4 v1 = make_float4(Rj, lc / Rj, 0.5f * sigma[ja], 2.0f * sqrtf(eps[ja]));
            if (slot == 0) {
                w0[lane] = v0; w0[64 + lane] = v0;
                w0[128 + lane] = v1; w0[192 + lane] = v1;
            } else {
                w1[lane] = v0; w1[64 + lane] = v1;
            }
        };
        fill(0, g.jbase);
        if (NSL > 1 && g.diag && g.phase == 0 && g.u_lim > 1) fill(NSL - 1, g.ibase + 64);
        wave_lds_fence();
        EnergyJ accj[NSL];
#pragma unroll
        for (int t = 0; t < NSL; ++t) accj[t] = EnergyJ{0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
        float e_c = 0.0f, e_g = 0.0f, e_lj = 0.0f;
        // sub-block u against j data (p0, p1): i-side sums, and the j-side terms
        // written (first) or added into c
        auto pair = [&](int u, const float4& p0, const float4& p1, bool ok, auto full, EnergyJ& c, bool first) {
            constexpr bool FULL = decltype(full)::value;
            const float dx = p0.x - xi[u], dy = p0.y - yi[u], dz = p0.z - zi[u];
            const float r2 = dx * dx + dy * dy + dz * dz;
            const bool valid = (FULL || ok) && (!EXT || r2 < ext.cut2);   // pair cutoff
            const float rinv = valid ? frsq(r2) : 0.0f;
            const float rinv2 = rinv * rinv;
            const float qq = qi[u] * p0.w;
            const float ec = qq * rinv;
            const float D2 = r2 * (Li[u] * p1.y);          // D log2(e)
            const float ex = __builtin_amdgcn_exp2f(-D2);   // exp(-D)
            const float f2 = __builtin_fmaf(Ri[u] * p1.x, ex, r2);
            const float finv = valid ? frsq(f2) : 0.0f;
            float eg = qq * finv;
            const float t = eg * finv * finv;               // qq / f^3
            // salt: the GB factor tau' becomes gsc = 1 - a exp(-kappa f) in the
            // energy and G1 = gsc - a kappa f exp(-kappa f) in its f-derivative
            float gsc = taup, G1 = taup;
            if (EXT) {
                const float f = f2 * finv;
                const float es = __builtin_amdgcn_exp2f(-ext.kl2e * f);
                gsc = __builtin_fmaf(ext.a, 1.0f - es, taup);
                G1 = __builtin_fmaf(-ext.ak * es, f, gsc);
                eg *= gsc;
            }
            const float sgr = (hsi[u] + p1.z) * rinv;
            const float s2 = sgr * sgr;
            const float s6 = s2 * s2 * s2;
            const float A = (sei[u] * p1.w) * s6;           // 4 eps_ij s^6
            const float B = A * s6;                         // 4 eps_ij s^12
            const float elj = B - A;
            const float uu = __builtin_fmaf(6.0f, B + elj, ec);
            const float w = EXT ? G1 * __builtin_fmaf(ex, -0.25f, 1.0f)
                                : __builtin_fmaf(ex, wq, taup);   // tau' (1 - exp(-D)/4)
            const float fs = __builtin_fmaf(-uu, rinv2, t * w);
            float gR = t * ex * __builtin_fmaf(D2, hl, 0.5f);
            if (EXT) gR *= G1;
            e_c += ec;
            e_g += eg;
            e_lj += elj;
            fxi[u] = __builtin_fmaf(fs, dx, fxi[u]);
            fyi[u] = __builtin_fmaf(fs, dy, fyi[u]);
            fzi[u] = __builtin_fmaf(fs, dz, fzi[u]);
            dRi[u] = __builtin_fmaf(gR, p1.x, dRi[u]);
            if (first) {
                c.x = -fs * dx; c.y = -fs * dy; c.z = -fs * dz; c.R = gR * Ri[u];
            } else {
                c.x = __builtin_fmaf(-fs, dx, c.x);
                c.y = __builtin_fmaf(-fs, dy, c.y);
                c.z = __builtin_fmaf(-fs, dz, c.z);
                c.R = __builtin_fmaf(gR, Ri[u], c.R);
            }
            if (GQ) {
                const float wqq = __builtin_fmaf(-gsc, finv, rinv);
                dqi[u] = __builtin_fmaf(wqq, p0.w, dqi[u]);
                c.q = first ? wqq * qi[u] : __builtin_fmaf(wqq, qi[u], c.q);
            }
        };
        auto rotate = [&](EnergyJ& a, const EnergyJ& c) {
            a.x = rot_add<EXT>(a.x, c.x);
            a.y = rot_add<EXT>(a.y, c.y);
            a.z = rot_add<EXT>(a.z, c.z);
            a.R = rot_add<EXT>(a.R, c.R);
            if (GQ) a.q = rot_add<EXT>(a.q, c.q);
        };
        auto kloop = [&](auto full, int k0, int k1) {
            constexpr bool FULL = decltype(full)::value;
            for (int k = k0; k < k1; ++k) {
                const int mu = lane + k + 1;             // 1 .. 127: the second copy past 63
                const int m = mu & 63;
                const float4 p0 = w0[mu], p1 = w0[128 + mu];
                EnergyJ c{0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
                for (int u = 0; u < NI; ++u)
                    if (FULL || u < g.u_lim)
                        pair(u, p0, p1, FULL || pair_ok<NI, EXT>(g, lane, k, m, li[u]), full, c, u == 0);
                rotate(accj[0], c);
            }
        };
        if constexpr (NI == 2) {
            if (g.diag) {
                // sub-task 1's tile: slot 1 in phase 0, slot 0 in phase 1
                const float4* const b1 = g.phase ? w0 : w1;
                const int c1o = g.phase ? 128 : 64;
                run_diag(g, lane, [&](int m0, int m1, bool ok0, bool ok1) {
                    EnergyJ c0{0.0f, 0.0f, 0.0f, 0.0f, 0.0f}, c1{0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
                    pair(0, w0[m0], w0[128 + m0], ok0, std::false_type{}, c0, true);
                    rotate(accj[0], c0);
                    if (g.u_lim > 1) {
                        pair(1, b1[m1], b1[c1o + m1], ok1, std::false_type{}, c1, true);
                        rotate(accj[NSL - 1], c1);
                    }
                });
            } else {
                run_item<NI, EXT>(g, kloop);
            }
        } else {
            run_item<NI, EXT>(g, kloop);
        }
        wave_lds_fence();
#pragma unroll
        for (int u = 0; u < NI; ++u) {
            if (u < g.u_lim && li[u] < g.n) {
                const int a = g.a0 + li[u];
                atomic_add_fx(&force_fx[a], to_fixed_f(fxi[u], FXF_FORCE, err));
                atomic_add_fx(&force_fx[ntot + a], to_fixed_f(fyi[u], FXF_FORCE, err));
                atomic_add_fx(&force_fx[2 * ntot + a], to_fixed_f(fzi[u], FXF_FORCE, err));
                atomic_add_fx(&dEdR_fx[a], to_fixed_f(EXT ? dRi[u] : dRi[u] * taup, FXF_FORCE, err));
                if (GQ) atomic_add_fx(&dEdq_fx[a], to_fixed_f(dqi[u] * sq_ke_in, FXF_FORCE, err));
            }
        }
        auto flush_j = [&](int jl, const EnergyJ& aj) {
            if (jl >= g.n) return;
            const int a = g.a0 + jl;
            atomic_add_fx(&force_fx[a], to_fixed_f(aj.x, FXF_FORCE, err));
            atomic_add_fx(&force_fx[ntot + a], to_fixed_f(aj.y, FXF_FORCE, err));
            atomic_add_fx(&force_fx[2 * ntot + a], to_fixed_f(aj.z, FXF_FORCE, err));
            atomic_add_fx(&dEdR_fx[a], to_fixed_f(EXT ? aj.R : aj.R * taup, FXF_FORCE, err));
            if (GQ) atomic_add_fx(&dEdq_fx[a], to_fixed_f(aj.q * sq_ke_in, FXF_FORCE, err));
        };
        flush_j(j_of_slot<EXT>(g, (lane + g.k1) & 63), accj[0]);
        if (NSL > 1 && g.diag && g.u_lim > 1)
            flush_j(g.ibase + 64 + ((lane + (g.phase ? 64 : 32)) & 63), accj[NSL - 1]);
        // per-lane energies to fixed point, summed over the wavefront as integers
        // and kept (lane 63) while the wavefront's items stay in one replica
        const long long sgb = wave_sum_i64_lane63(to_fixed_f(EXT ? -e_g : -taup * e_g, FXF_ENERGY, err));
        const long long sc = wave_sum_i64_lane63(to_fixed_f(e_c, FXF_ENERGY, err));
        const long long slj = wave_sum_i64_lane63(to_fixed_f(e_lj, FXF_ENERGY, err));
        if (g.rep != e_rep) {
            flush_e();
            e_rep = g.rep;
        }
        e_sum[0] += sgb;
        e_sum[1] += sc;
        e_sum[2] += slj;
    }
    flush_e();
}

// ------------------------------------------------- chain rule through psi
// F_i += g (x_j - x_i)/r,  g = c_i dh(r; rt_i, s_j)/dr + c_j dh(r; rt_j, s_i)/dr,
// c = (dE/dR)(dR/dpsi)(rho~/2).  Distant spheres: dh/dr = -(s^3/r^5) Q(s^2/r^2),
// so g/r = -(c_i s_j^3 Q_ij + c_j s_i^3 Q_ji) / r^6.
// With RHO also the pair part of dE/drho:
//   i: c_i dh_ij/drt + S_i c_j dh_ji/ds,   j: c_j dh_ji/drt + S_j c_i dh_ij/ds.
// j tile in LDS: {x, y, z, c}, {rt, s, m, sx}, {s^2, s^3, S, -}.
struct ChainJ {
    float x, y, z, r;
};

template <int NI, bool RHO, bool EXT>
__global__ __launch_bounds__(256) void k_chain_pair(
    const int2* __restrict__ items, int n_items, const int32_t* __restrict__ n_dev,
    const int32_t* __restrict__ atom_off, int ntot,
    const float* __restrict__ xyz, const float* __restrict__ rho,
    const float* __restrict__ screen, const float* __restrict__ cc, float offset, PairExt ext,
    int64_t* __restrict__ force_fx, int64_t* __restrict__ dEdrho_fx, uint32_t* __restrict__ err)
{
    constexpr int NSL = NI == 2 ? 2 : 1;
    extern __shared__ float4 lds_dyn[];          // j tiles: [waves in the group][NSL][3][64]
    auto lds = reinterpret_cast<float4 (*)[NSL][3][64]>(lds_dyn);
    const int lane = threadIdx.x & 63, wv = wave_in_group();
    const int stride = gridDim.x * (blockDim.x >> 6);
    const float ixmax = 1.0f / HCT_FAR_XMAX;
    if (n_dev) n_items = n_dev[0];                // a packed list: its device count
    for (int it = logical_wave(); it < n_items; it += stride) {
        const ItemGeom g = item_geom<NI, EXT>(items[it], atom_off, ext);
        float xi[NI], yi[NI], zi[NI], rti[NI], si[NI], ci[NI], Si[NI], mi[NI], sxi[NI], s2i[NI], s3i[NI];
        float fxi[NI], fyi[NI], fzi[NI], dri[NI];
        int li[NI];
#pragma unroll
        for (int u = 0; u < NI; ++u) {
            li[u] = item_li<NI>(g, u, lane);
            const int a = g.a0 + min(li[u], g.n - 1);
            xi[u] = xyz[a]; yi[u] = xyz[ntot + a]; zi[u] = xyz[2 * ntot + a];
            rti[u] = rho[a] - offset;
            Si[u] = screen[a];
            si[u] = Si[u] * rti[u];
            ci[u] = cc[a];
            mi[u] = fmaxf(rti[u], si[u]);
            sxi[u] = si[u] * ixmax;
            s2i[u] = si[u] * si[u];
            s3i[u] = s2i[u] * si[u];
            fxi[u] = fyi[u] = fzi[u] = dri[u] = 0.0f;
        }
        auto fill = [&](int slot, int tb) {
            const int ja = g.a0 + j_fill<EXT>(g, tb, lane);
            const float rt = rho[ja] - offset, S = screen[ja], s = S * rt;
            lds[wv][slot][0][lane] = make_float4(xyz[ja], xyz[ntot + ja], xyz[2 * ntot + ja], cc[ja]);
            lds[wv][slot][1][lane] = make_float4(rt, s, fmaxf(rt, s), s * ixmax);
            lds[wv][slot][2][lane] = make_float4(s * s, s * s * s, S, 0.0f);
        };
        fill(0, g.jbase);
        if (NSL > 1 && g.diag && g.phase == 0 && g.u_lim > 1) fill(NSL - 1, g.ibase + 64);
        wave_lds_fence();
        ChainJ accj[NSL];
#pragma unroll
        for (int t = 0; t < NSL; ++t) accj[t] = ChainJ{0.0f, 0.0f, 0.0f, 0.0f};
        auto pair = [&](int u, const float4& p0, const float4& p1, const float4& p2, bool ok, auto full,
                        ChainJ& c, bool first) {
            constexpr bool FULL = decltype(full)::value;
            const float dx = p0.x - xi[u], dy = p0.y - yi[u], dz = p0.z - zi[u];
            float r2 = dx * dx + dy * dy + dz * dz;
            if (!FULL) r2 = ok ? r2 : FAR_R2;
            if (EXT) r2 = r2 < ext.rgb2 ? r2 : FAR_R2;      // descreening cutoff
            const float rinv = frsq(r2);
            const float r = r2 * rinv;
            const float rinv2 = rinv * rinv;
            float fs;
            if (!RHO) {
                const float Qij = poly_Q(p2.x * rinv2), Qji = poly_Q(s2i[u] * rinv2);
                const float G = __builtin_fmaf(p0.w * s3i[u], Qji, ci[u] * (p2.y * Qij));
                fs = -G * (rinv2 * rinv2 * rinv2);
                if (!both_far(r, mi[u], p1.z, sxi[u], p1.w)) {
                    const float dij = (r + p1.y <= rti[u]) ? 0.0f : hct_dr_closed(r, rinv, rti[u], p1.y);
                    const float dji = (r + si[u] <= p1.x) ? 0.0f : hct_dr_closed(r, rinv, p1.x, si[u]);
                    fs = (ci[u] * dij + p0.w * dji) * rinv;
                }
            } else {
                float dr_ij, drt_ij, ds_ij, dr_ji, drt_ji, ds_ji;
                hct_grad3(r, rinv, rti[u], p1.y, dr_ij, drt_ij, ds_ij);
                hct_grad3(r, rinv, p1.x, si[u], dr_ji, drt_ji, ds_ji);
                fs = (ci[u] * dr_ij + p0.w * dr_ji) * rinv;
                dri[u] += ci[u] * drt_ij + Si[u] * p0.w * ds_ji;
                const float cr = p0.w * drt_ji + p2.z * ci[u] * ds_ij;
                c.r = first ? cr : c.r + cr;
            }
            fxi[u] = __builtin_fmaf(fs, dx, fxi[u]);
            fyi[u] = __builtin_fmaf(fs, dy, fyi[u]);
            fzi[u] = __builtin_fmaf(fs, dz, fzi[u]);
            if (first) {
                c.x = -fs * dx; c.y = -fs * dy; c.z = -fs * dz;
            } else {
                c.x = __builtin_fmaf(-fs, dx, c.x);
                c.y = __builtin_fmaf(-fs, dy, c.y);
                c.z = __builtin_fmaf(-fs, dz, c.z);
            }
        };
        auto rotate = [&](ChainJ& a, const ChainJ& c) {
            a.x = rot_add<EXT>(a.x, c.x);
            a.y = rot_add<EXT>(a.y, c.y);
            a.z = rot_add<EXT>(a.z, c.z);
            if (RHO) a.r = rot_add<EXT>(a.r, c.r);
        };
        auto kloop = [&](auto full, int k0, int k1) {
            constexpr bool FULL = decltype(full)::value;
            for (int k = k0; k < k1; ++k) {
                const int m = (lane + k + 1) & 63;
                const float4 p0 = lds[wv][0][0][m], p1 = lds[wv][0][1][m], p2 = lds[wv][0][2][m];
                ChainJ c{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
                for (int u = 0; u < NI; ++u)
                    if (FULL || u < g.u_lim)
                        pair(u, p0, p1, p2, FULL || pair_ok<NI, EXT>(g, lane, k, m, li[u]), full, c, u == 0);
                rotate(accj[0], c);
            }
        };
        if constexpr (NI == 2) {
            if (g.diag) {
                const int s1 = g.phase ? 0 : NSL - 1;
                run_diag(g, lane, [&](int m0, int m1, bool ok0, bool ok1) {
                    ChainJ c0{0.0f, 0.0f, 0.0f, 0.0f}, c1{0.0f, 0.0f, 0.0f, 0.0f};
                    pair(0, lds[wv][0][0][m0], lds[wv][0][1][m0], lds[wv][0][2][m0], ok0, std::false_type{}, c0, true);
                    rotate(accj[0], c0);
                    if (g.u_lim > 1) {
                        pair(1, lds[wv][s1][0][m1], lds[wv][s1][1][m1], lds[wv][s1][2][m1], ok1, std::false_type{},
                             c1, true);
                        rotate(accj[NSL - 1], c1);
                    }
                });
            } else {
                run_item<NI, EXT>(g, kloop);
            }
        } else {
            run_item<NI, EXT>(g, kloop);
        }
        wave_lds_fence();
#pragma unroll
        for (int u = 0; u < NI; ++u) {
            if (u < g.u_lim && li[u] < g.n) {
                const int a = g.a0 + li[u];
                atomic_add_fx(&force_fx[a], to_fixed_f(fxi[u], FXF_FORCE, err));
                atomic_add_fx(&force_fx[ntot + a], to_fixed_f(fyi[u], FXF_FORCE, err));
                atomic_add_fx(&force_fx[2 * ntot + a], to_fixed_f(fzi[u], FXF_FORCE, err));
                if (RHO) atomic_add_fx(&dEdrho_fx[a], to_fixed_f(dri[u], FXF_FORCE, err));
            }
        }
        auto flush_j = [&](int jl, const ChainJ& aj) {
            if (jl >= g.n) return;
            const int a = g.a0 + jl;
            atomic_add_fx(&force_fx[a], to_fixed_f(aj.x, FXF_FORCE, err));
            atomic_add_fx(&force_fx[ntot + a], to_fixed_f(aj.y, FXF_FORCE, err));
            atomic_add_fx(&force_fx[2 * ntot + a], to_fixed_f(aj.z, FXF_FORCE, err));
            if (RHO) atomic_add_fx(&dEdrho_fx[a], to_fixed_f(aj.r, FXF_FORCE, err));
        };
        flush_j(j_of_slot<EXT>(g, (lane + g.k1) & 63), accj[0]);
        if (NSL > 1 && g.diag && g.u_lim > 1)
            flush_j(g.ibase + 64 + ((lane + (g.phase ? 64 : 32)) & 63), accj[NSL - 1]);
    }
}

// ------------------------------------------------------------- packing
// With both cutoffs the pair passes run, per list and radius, the list's
// intra-block items (a fixed prefix) followed by packed items built at every
// evaluation from the current positions.

// Per-tile bounding boxes: one wavefront per tile, min / max over its atoms.
// Also resets the eight list counters to their intra-block item counts (the
// packing kernels run after).
struct CountInit {
    int32_t v[8];
};

__global__ __launch_bounds__(256) void k_tile_boxes(
    const int2* __restrict__ tiles, int n_tiles, const int32_t* __restrict__ atom_off, int ntot,
    const float* __restrict__ xyz, float4* __restrict__ box, int32_t* __restrict__ counts,
    CountInit init)
{
    if (blockIdx.x == 0 && threadIdx.x < 8) counts[threadIdx.x] = init.v[threadIdx.x];
    const int t = blockIdx.x * (blockDim.x >> 6) + wave_in_group();
    if (t >= n_tiles) return;
    const int lane = threadIdx.x & 63;
    const int2 tl = tiles[t];
    const int a0 = atom_off[tl.x], n = atom_off[tl.x + 1] - a0;
    const int li = min(tl.y * 64 + lane, n - 1);        // the tail repeats the last atom
    const int a = a0 + li;
    float lo[3], hi[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) lo[d] = hi[d] = xyz[(int64_t)d * ntot + a];
    for (int off = 32; off > 0; off >>= 1) {
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            lo[d] = fminf(lo[d], __shfl_xor(lo[d], off, 64));
            hi[d] = fmaxf(hi[d], __shfl_xor(hi[d], off, 64));
        }
    }
    if (lane == 0) {
        box[2 * t] = make_float4(lo[0], lo[1], lo[2], 0.0f);
        box[2 * t + 1] = make_float4(hi[0], hi[1], hi[2], 0.0f);
    }
}

// Packing, in two passes.  Every I block (rep, A) with tiles after it owns
// the packed tiles P0 .. P0 + (T - t1) - 1 (t1: the first tile after the
// block), as many as it has tiles after it, and their 64 J slots each.
//  k_pack_atoms: one workgroup per I block, its PACK_WAVES wavefronts scanning
//    the block's windows of up to PACK_WINDOW tiles (one window each per round):
//    the tiles whose box comes within rc of the block's box, then their atoms
//    within rc of it, written to the block's slots in window, tile and lane
//    order (each window after the counts of the windows before it).  Where
//    every atom lands depends on the coordinates alone, so the packed items
//    (and the FP32 sums over them) are the same at every evaluation of the
//    same positions.
//  k_pack_items: one lane per block; its atoms form ceil(count / 64) packed
//    items {rep | ITEM_PACKED << 30, P}, pk_hdr[P] = A << 7 | nj, appended to
//    the list after its intra-block items (in an order that changes no
//    result); the count is cleared for the next evaluation.
// Every pair the packing drops is farther apart than rc, so the kernels'
// cutoff would have made its terms exact zeros; the order of the J atoms and
// of the items changes no result (fixed-point sums).
__device__ __forceinline__ float box_gap2(float4 alo, float4 ahi, float4 blo, float4 bhi) {
    const float dx = fmaxf(0.0f, fmaxf(alo.x - bhi.x, blo.x - ahi.x));
    const float dy = fmaxf(0.0f, fmaxf(alo.y - bhi.y, blo.y - ahi.y));
    const float dz = fmaxf(0.0f, fmaxf(alo.z - bhi.z, blo.z - ahi.z));
    return dx * dx + dy * dy + dz * dz;
}

constexpr int PACK_BATCH = 4;       // tiles whose atoms are loaded together

// Outputs of one radius: rc^2, the blocks' atom counts, the J slots, and (items
// pass) the run list, its count and the packed tiles' headers.
struct PackOut {
    float rc2;
    int32_t* blk_count;
    int32_t* pk_j;
    int2* items;
    int32_t* count;
    int32_t* pk_hdr;
};

// NK = 2 packs the lists of both radii (descreening and energy passes on the
// same blocking) in one scan: tiles tested against the larger radius, atoms
// against each.
constexpr int PACK_WAVES = 8;       // wavefronts of a packing workgroup (windows per round)

template <int NK>
__global__ __launch_bounds__(64 * PACK_WAVES) void k_pack_atoms(
    const int4* __restrict__ win, const int32_t* __restrict__ blk_win, int n_iblk, int ni,
    const int32_t* __restrict__ atom_off, const int32_t* __restrict__ tile_base,
    const float4* __restrict__ box, const float* __restrict__ xyz, int ntot, PackOut o0, PackOut o1)
{
    __shared__ unsigned long long s_mask[NK][PACK_WAVES][PACK_WINDOW];
    __shared__ int s_tile[PACK_WAVES][PACK_WINDOW];
    __shared__ int s_tot[NK][PACK_WAVES];
    const int lane = threadIdx.x & 63, wv = wave_in_group(), nw = (int)(blockDim.x >> 6);
    const int bi = blockIdx.x;                         // one workgroup per I block
    const PackOut* out[2] = {&o0, &o1};
    float rc2[NK];
    float rt2 = 0.0f;
#pragma unroll
    for (int v = 0; v < NK; ++v) {
        rc2[v] = out[v]->rc2;
        rt2 = fmaxf(rt2, rc2[v]);
    }
    const int w0 = blk_win[bi], w1 = blk_win[bi + 1];
    // {block, A << 16 | first tile, the block's first packed tile, replica}:
    // block, tile range and replica from the first window
    const int4 wd0 = win[w0];
    const int rep = wd0.w, A = (int)((unsigned)wd0.y >> 16);
    const int a0 = atom_off[rep], n = atom_off[rep + 1] - a0;
    const int T = (n + 63) >> 6, tb = tile_base[rep];
    const int t0 = A * ni, t1 = min(T, t0 + ni);
    float4 lo = box[2 * (tb + t0)], hi = box[2 * (tb + t0) + 1];
    for (int t = t0 + 1; t < t1; ++t) {
        const float4 l = box[2 * (tb + t)], h = box[2 * (tb + t) + 1];
        lo = make_float4(fminf(lo.x, l.x), fminf(lo.y, l.y), fminf(lo.z, l.z), 0.0f);
        hi = make_float4(fmaxf(hi.x, h.x), fmaxf(hi.y, h.y), fmaxf(hi.z, h.z), 0.0f);
    }
    const unsigned long long below = (1ull << lane) - 1ull;
    int done[NK];                                      // atoms of this block placed so far, per radius
#pragma unroll
    for (int v = 0; v < NK; ++v) done[v] = 0;
    constexpr int NQ = (PACK_WINDOW + 63) / 64;
    // rounds of nw windows: wavefront w scans window w0 + nw r + w; the
    // round's counts are met in LDS and each window writes after the windows
    // before it, so the slots follow window, tile and lane order
    for (int wr = w0; wr < w1; wr += nw) {
        const int wi = wr + wv;
        int nn = 0, total[NK];
#pragma unroll
        for (int v = 0; v < NK; ++v) total[v] = 0;
        if (wi < w1) {
            const int c0 = win[wi].y & 0xFFFF;
            // the window's tiles, 64 to a ballot word (lane l of word q: tile c0 + 64 q + l)
            unsigned long long nmq[NQ];
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                const int t = c0 + 64 * q + lane;
                bool near = false;
                if (64 * q + lane < PACK_WINDOW && t < T)
                    near = box_gap2(lo, hi, box[2 * (tb + t)], box[2 * (tb + t) + 1]) < rt2;
                nmq[q] = __ballot(near);
            }
            int q = 0;
            unsigned long long nm = nmq[0];
            auto next_tile = [&]() -> int {            // next near tile of the window, or -1
                while (!nm && q + 1 < NQ) nm = nmq[++q];
                if (!nm) return -1;
                const int b = c0 + 64 * q + __ffsll((long long)nm) - 1;
                nm &= nm - 1ull;
                return b;
            };
            for (;;) {
                int bt[PACK_BATCH];
                float x[PACK_BATCH], y[PACK_BATCH], z[PACK_BATCH];
                bool any = false;
#pragma unroll
                for (int k = 0; k < PACK_BATCH; ++k) {
                    bt[k] = next_tile();
                    if (bt[k] >= 0) {
                        any = true;
                        const int jl = min(bt[k] * 64 + lane, n - 1);
                        x[k] = xyz[a0 + jl]; y[k] = xyz[ntot + a0 + jl]; z[k] = xyz[2 * ntot + a0 + jl];
                    }
                }
                if (!any) break;
#pragma unroll
                for (int k = 0; k < PACK_BATCH; ++k) {
                    if (bt[k] < 0) break;
                    const float dx = fmaxf(0.0f, fmaxf(lo.x - x[k], x[k] - hi.x));
                    const float dy = fmaxf(0.0f, fmaxf(lo.y - y[k], y[k] - hi.y));
                    const float dz = fmaxf(0.0f, fmaxf(lo.z - z[k], z[k] - hi.z));
                    const float d2 = dx * dx + dy * dy + dz * dz;
                    const bool in = bt[k] * 64 + lane < n;
                    unsigned long long am[NK];
                    unsigned long long anym = 0;
#pragma unroll
                    for (int v = 0; v < NK; ++v) {
                        am[v] = __ballot(in && d2 < rc2[v]);
                        anym |= am[v];
                    }
                    if (anym) {
                        if (lane == 0) {
#pragma unroll
                            for (int v = 0; v < NK; ++v) s_mask[v][wv][nn] = am[v];
                            s_tile[wv][nn] = bt[k];
                        }
                        ++nn;
#pragma unroll
                        for (int v = 0; v < NK; ++v) total[v] += __popcll(am[v]);
                    }
                }
            }
        }
        if (lane == 0) {
#pragma unroll
            for (int v = 0; v < NK; ++v) s_tot[v][wv] = total[v];
        }
        __syncthreads();
#pragma unroll
        for (int v = 0; v < NK; ++v) {
            int before = done[v], all = done[v];
            for (int u = 0; u < nw; ++u) {
                if (u < wv) before += s_tot[v][u];
                all += s_tot[v][u];
            }
            if (total[v] > 0) {
                int32_t* dst = out[v]->pk_j + (int64_t)wd0.z * 64 + before;
                for (int k = 0; k < nn; ++k) {
                    const unsigned long long am = s_mask[v][wv][k];
                    if ((am >> lane) & 1ull) dst[__popcll(am & below)] = s_tile[wv][k] * 64 + lane;
                    dst += __popcll(am);
                }
            }
            done[v] = all;
        }
        __syncthreads();                               // the next round reuses s_mask, s_tile, s_tot
    }
    if (threadIdx.x == 0) {
#pragma unroll
        for (int v = 0; v < NK; ++v) out[v]->blk_count[bi] = done[v];
    }
}

// One wavefront per radius and 64 blocks (NK wavefronts per workgroup).
template <int NK>
__global__ __launch_bounds__(64 * NK) void k_pack_items(
    const int2* __restrict__ iblk, const int32_t* __restrict__ blk_p0, int n_iblk, PackOut o0, PackOut o1)
{
    const int lane = threadIdx.x & 63;
    const int w = blockIdx.x * 64 + lane;
    const PackOut& o = (NK == 2 && (threadIdx.x >> 6)) ? o1 : o0;
    int2 ib = make_int2(0, 0);
    int p0 = 0, cnt = 0;
    if (w < n_iblk) {
        ib = iblk[w];
        p0 = blk_p0[w];
        cnt = o.blk_count[w];
        o.blk_count[w] = 0;
    }
    const int nt = (cnt + 63) >> 6;
    int pre = nt;                                  // inclusive prefix over the wavefront
    for (int d = 1; d < 64; d <<= 1) {
        const int t = __shfl_up(pre, d, 64);
        if (lane >= d) pre += t;
    }
    const int total = __shfl(pre, 63, 64);
    if (total == 0) return;
    int base = 0;
    if (lane == 63) base = atomicAdd(o.count, total);
    base = __shfl(base, 63, 64);
    // the wavefront writes block L's items together, block by block
    for (int L = 0; L < 64; ++L) {
        const int ntL = __shfl(nt, L, 64);
        if (ntL == 0) continue;
        const int slot0 = base + __shfl(pre, L, 64) - ntL;
        const int cntL = __shfl(cnt, L, 64), repL = __shfl(ib.x, L, 64), AL = __shfl(ib.y, L, 64);
        const int p0L = __shfl(p0, L, 64);
        for (int p = lane; p < ntL; p += 64) {
            o.items[slot0 + p] = make_int2(repL | (ITEM_PACKED << 30), p0L + p);
            o.pk_hdr[p0L + p] = (AL << 7) | min(64, cntL - 64 * p);
        }
    }
}

int grid_for(const gbr_ctx* c, int n_items) {
    const int W = c->shape.waves_per_group;
    int want = (n_items + W - 1) / W;
    int cap = c->n_cu * c->shape.groups_per_cu;
    int g = want < cap ? want : cap;
    if (g < 8) return g < 1 ? 1 : g;
    return (g + 7) & ~7;   // multiple of 8 for the XCD remapping
}

// Dynamic LDS of a pair kernel: the j tiles of the group's own wavefronts
// (comps float4 per atom, two tiles per wavefront at NI = 2), so that groups
// of fewer wavefronts take less LDS and more of them fit a CU.
size_t pair_lds(int waves, int ni, int comps) {
    return (size_t)waves * (ni == 2 ? 2 : 1) * comps * 64 * sizeof(float4);
}

// The energy pass: slot 0 holds its two components twice (2 x 128 float4).
size_t energy_lds(int waves, int ni) {
    return (size_t)waves * (256 + (ni == 2 ? 128 : 0)) * sizeof(float4);
}

// Nothing to launch: the timing events still get recorded (an empty interval).
hipError_t no_launch(hipStream_t s, const LaunchEvents& ev) {
    if (ev.start) (void)hipEventRecord(ev.start, s);
    if (ev.stop) (void)hipEventRecord(ev.stop, s);
    return hipSuccess;
}

const PairList& list_for(const gbr_ctx* c, int ni) {
    switch (ni) {
        case 1: return c->lists[0];
        case 2: return c->lists[1];
        case 4: return c->lists[2];
        default: return c->lists[3];
    }
}

}  // namespace

namespace gbr {

// kind: the packed lists of radius rgbmax (0, descreening passes) or cut (1).
static PairExt make_pair_ext(const gbr_ctx* c, const PairList& L, int kind) {
    const gbr_gb_params& p = c->prm;
    PairExt e;
    e.kl2e = (float)(p.kappa * 1.4426950408889634);
    e.a = (float)(p.eps_in / p.eps_out);
    e.ak = (float)(p.eps_in / p.eps_out * p.kappa);
    e.cut2 = p.cut > 0 ? (float)(p.cut * p.cut) : FLT_MAX;
    e.rgb2 = p.rgbmax > 0 ? (float)(p.rgbmax * p.rgbmax) : FLT_MAX;
    e.pk_hdr = c->packed ? L.pk_hdr[kind] : nullptr;
    e.pk_j = c->packed ? L.pk_j[kind] : nullptr;
    return e;
}

static bool uses_ext(const gbr_ctx* c) {
    return c->prm.kappa > 0 || c->prm.cut > 0 || c->prm.rgbmax > 0;
}

hipError_t launch_pack(const gbr_ctx* c, const float* xyz, hipStream_t s) {
    if (!c->packed) return hipSuccess;
    CountInit init;
    for (int k = 0; k < 4; ++k)
        for (int v = 0; v < 2; ++v) init.v[2 * k + v] = c->lists[k].n_intra;
    hipLaunchKernelGGL(k_tile_boxes, dim3((c->n_tiles + 3) / 4), dim3(256), 0, s, c->tiles, c->n_tiles,
                       c->atom_off, c->n_atoms, xyz, c->tile_box, c->pack_count, init);
    // the tile boxes' FP32 bounds are exact (min / max of the stored
    // coordinates); the margin covers the rounding of the kernels' own r^2
    const double rc[2] = {c->prm.rgbmax * (1.0 + 1e-5) + 1e-4, c->prm.cut * (1.0 + 1e-5) + 1e-4};
    auto pack_out = [&](const PairList& L, int v) {
        return PackOut{(float)(rc[v] * rc[v]), L.blk_count[v], L.pk_j[v], L.run[v], L.n_run[v], L.pk_hdr[v]};
    };
    auto idx_of = [](int ni) { return ni == 1 ? 0 : ni == 2 ? 1 : ni == 4 ? 2 : 3; };
    const int ib = idx_of(c->ni_born), ic = idx_of(c->ni_chain), ie = idx_of(c->ni_energy);
    // lists in use: {list, radius}; a list used with both radii is packed in one scan
    bool need[4][2] = {};
    need[ib][0] = need[ic][0] = true;
    need[ie][1] = true;
    for (int k = 0; k < 4; ++k) {
        const PairList& L = c->lists[k];
        if (L.n_iblk == 0 || !(need[k][0] || need[k][1])) continue;
        const dim3 ga(L.n_iblk), gi((L.n_iblk + 63) / 64);
        if (need[k][0] && need[k][1]) {
            const PackOut o0 = pack_out(L, 0), o1 = pack_out(L, 1);
            hipLaunchKernelGGL(k_pack_atoms<2>, ga, dim3(64 * PACK_WAVES), 0, s, L.win, L.blk_win, L.n_iblk, L.ni, c->atom_off,
                               c->tile_base, c->tile_box, xyz, c->n_atoms, o0, o1);
            hipLaunchKernelGGL(k_pack_items<2>, gi, dim3(128), 0, s, L.iblk, L.blk_p0, L.n_iblk, o0, o1);
        } else {
            const PackOut o = pack_out(L, need[k][0] ? 0 : 1);
            hipLaunchKernelGGL(k_pack_atoms<1>, ga, dim3(64 * PACK_WAVES), 0, s, L.win, L.blk_win, L.n_iblk, L.ni, c->atom_off,
                               c->tile_base, c->tile_box, xyz, c->n_atoms, o, o);
            hipLaunchKernelGGL(k_pack_items<1>, gi, dim3(64), 0, s, L.iblk, L.blk_p0, L.n_iblk, o, o);
        }
    }
    return hipGetLastError();
}

hipError_t launch_born_pair(const gbr_ctx* c, const float* xyz, const float* rho,
                            const float* screen, hipStream_t s, LaunchEvents ev)
{
    const PairList& L = list_for(c, c->ni_born);
    if (L.n_items == 0) return no_launch(s, ev);
    dim3 grid(grid_for(c, L.n_items)), block(64 * c->shape.waves_per_group);
    const int2* items = c->packed ? L.run[0] : L.items;
    const int32_t* n_dev = c->packed ? L.n_run[0] : nullptr;
    const float off = (float)c->prm.offset;
    const PairExt pe = make_pair_ext(c, L, 0);
    const bool ext = uses_ext(c);
#define GBR_BORN(NI, EX) hipExtLaunchKernelGGL((k_born_pair<NI, EX>), grid, block, \
        pair_lds(c->shape.waves_per_group, NI, 2), s, ev.start, ev.stop, 0, \
        items, L.n_items, n_dev, c->atom_off, c->n_atoms, xyz, rho, screen, off, pe, c->psi_fx, c->err, 0)
    switch (L.ni) {
        case 1: if (ext) GBR_BORN(1, true); else GBR_BORN(1, false); break;
        case 2: if (ext) GBR_BORN(2, true); else GBR_BORN(2, false); break;
        case 4: if (ext) GBR_BORN(4, true); else GBR_BORN(4, false); break;
        default: if (ext) GBR_BORN(8, true); else GBR_BORN(8, false); break;
    }
#undef GBR_BORN
    return hipGetLastError();
}

hipError_t launch_born_pair_gen(const gbr_gb_params& p, int n_rep, int max_tiles, const int32_t* atom_off,
                                int n_atoms, int n_cu, const float* xyz, const float* rho,
                                const float* screen, int64_t* psi_fx, uint32_t* err, hipStream_t s)
{
    const int64_t n_items = (int64_t)n_rep * max_tiles * max_tiles;   // checked < 2^31 by the caller
    const int64_t want = (n_items + 3) / 4;
    int g = (int)std::min<int64_t>(want, (int64_t)n_cu * 8);
    if (g >= 8) g = (g + 7) & ~7;               // multiple of 8 for the XCD remapping
    PairExt pe{};
    pe.rgb2 = p.rgbmax > 0 ? (float)(p.rgbmax * p.rgbmax) : FLT_MAX;
    const float off = (float)p.offset;
    if (p.rgbmax > 0)
        hipLaunchKernelGGL((k_born_pair<1, true, true>), dim3(g), dim3(256), pair_lds(4, 1, 2), s, (const int2*)nullptr,
                           (int)n_items, (const int32_t*)nullptr, atom_off, n_atoms, xyz, rho, screen, off, pe,
                           psi_fx, err, max_tiles);
    else
        hipLaunchKernelGGL((k_born_pair<1, false, true>), dim3(g), dim3(256), pair_lds(4, 1, 2), s, (const int2*)nullptr,
                           (int)n_items, (const int32_t*)nullptr, atom_off, n_atoms, xyz, rho, screen, off, pe,
                           psi_fx, err, max_tiles);
    return hipGetLastError();
}

hipError_t launch_energy_pair(const gbr_ctx* c, const float* xyz, const float* q,
                              const float* R, const float* sigma, const float* eps,
                              int64_t* force_fx, int64_t* dEdq_fx,
                              hipStream_t s, LaunchEvents ev)
{
    const PairList& L = list_for(c, c->ni_energy);
    if (L.n_items == 0) return no_launch(s, ev);
    dim3 grid(grid_for(c, L.n_items)), block(64 * c->shape.waves_per_group);
    const int2* items = c->packed ? L.run[1] : L.items;
    const int32_t* n_dev = c->packed ? L.n_run[1] : nullptr;
    const float sq = (float)sqrt(c->prm.k_e / c->prm.eps_in);
    const float taup = (float)((1.0 / c->prm.eps_in - 1.0 / c->prm.eps_out) * c->prm.eps_in);
    const PairExt pe = make_pair_ext(c, L, 1);
#define GBR_EN(NI, GQ, EX) hipExtLaunchKernelGGL((k_energy_pair<NI, GQ, EX>), grid, block, \
        energy_lds(c->shape.waves_per_group, NI), s, ev.start, \
        ev.stop, 0, items, L.n_items, n_dev, c->atom_off, c->n_atoms, xyz, q, R, sigma, eps, sq, taup, pe, \
        force_fx, c->dEdR_fx, c->e_stripe, dEdq_fx, c->err)
#define GBR_EN2(NI, GQ) if (uses_ext(c)) GBR_EN(NI, GQ, true); else GBR_EN(NI, GQ, false)
    const bool gq = dEdq_fx != nullptr;
    switch (L.ni) {
        case 1: if (gq) { GBR_EN2(1, true); } else { GBR_EN2(1, false); } break;
        case 2: if (gq) { GBR_EN2(2, true); } else { GBR_EN2(2, false); } break;
        case 4: if (gq) { GBR_EN2(4, true); } else { GBR_EN2(4, false); } break;
        default: if (gq) { GBR_EN2(8, true); } else { GBR_EN2(8, false); } break;
    }
#undef GBR_EN2
#undef GBR_EN
    return hipGetLastError();
}

hipError_t launch_chain_pair(const gbr_ctx* c, const float* xyz, const float* rho,
                             const float* screen, int64_t* force_fx, int64_t* dEdrho_fx,
                             hipStream_t s, LaunchEvents ev)
{
    const PairList& L = list_for(c, c->ni_chain);
    if (L.n_items == 0) return no_launch(s, ev);
    dim3 grid(grid_for(c, L.n_items)), block(64 * c->shape.waves_per_group);
    const int2* items = c->packed ? L.run[0] : L.items;
    const int32_t* n_dev = c->packed ? L.n_run[0] : nullptr;
    const float off = (float)c->prm.offset;
    const PairExt pe = make_pair_ext(c, L, 0);
#define GBR_CH(NI, RH, EX) hipExtLaunchKernelGGL((k_chain_pair<NI, RH, EX>), grid, block, \
        pair_lds(c->shape.waves_per_group, NI, 3), s, ev.start, \
        ev.stop, 0, items, L.n_items, n_dev, c->atom_off, c->n_atoms, xyz, rho, screen, c->chain_c, off, pe, \
        force_fx, dEdrho_fx, c->err)
#define GBR_CH2(NI, RH) if (uses_ext(c)) GBR_CH(NI, RH, true); else GBR_CH(NI, RH, false)
    const bool rh = dEdrho_fx != nullptr;
    switch (L.ni) {
        case 1: if (rh) { GBR_CH2(1, true); } else { GBR_CH2(1, false); } break;
        case 2: if (rh) { GBR_CH2(2, true); } else { GBR_CH2(2, false); } break;
        case 4: if (rh) { GBR_CH2(4, true); } else { GBR_CH2(4, false); } break;
        default: if (rh) { GBR_CH2(8, true); } else { GBR_CH2(8, false); } break;
    }
#undef GBR_CH2
#undef GBR_CH
    return hipGetLastError();
}

}  // namespace gbr
