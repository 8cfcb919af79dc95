// gbr_device.h -- device helpers shared by the library's kernels:
// fixed-point accumulation, wavefront reductions, the counter-based RNG, and
// the FP32 descreening term with its derivatives.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gbremd.h"
#include "hct_poly.h"

#define GBR_WAVE 64

namespace gbr {

// ---------------------------------------------------------------- constants
constexpr double KB = 0.001987204259;     // kcal/(mol K), CODATA 2018 R / 4184 J/kcal
constexpr double FARADAY = 23.0605480;    // kcal/(mol V), CODATA 2018 F / 4184 J/kcal
constexpr double LN10 = 2.302585092994045684;
constexpr double ACC_CONV = 418.4;        // 1 kcal/(mol A amu) in A/ps^2
constexpr double FX_FORCE = 1099511627776.0;   // 2^40
constexpr double FX_ENERGY = 4294967296.0;     // 2^32
constexpr double INV_FX_FORCE = 1.0 / FX_FORCE;
constexpr double INV_FX_ENERGY = 1.0 / FX_ENERGY;
constexpr float FXF_FORCE = 1099511627776.0f;  // the same scales as floats
constexpr float FXF_ENERGY = 4294967296.0f;

enum Stream : uint32_t { STREAM_O = 1, STREAM_MCPH = 2, STREAM_MCRED = 3, STREAM_EX = 4 };



// ------------------------------------------------------------ fixed point
__device__ __forceinline__ void raise_error(uint32_t* err, uint32_t bits) {
    __hip_atomic_fetch_or(err, bits, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// round(v * scale) with saturation reported in the error word.
__device__ __forceinline__ long long to_fixed(double v, double scale, uint32_t* err) {
    double s = v * scale;
    if (!(fabs(s) < 4.6116860184273879e18)) {   // 2^62
        raise_error(err, (v == v && fabs(v) <= 1.7976931348623157e308) ? GBR_ERR_OVERFLOW
                                                                        : GBR_ERR_NONFINITE);
        return 0;
    }
    return (long long)__builtin_rint(s);
}

// The same for an FP32 value and a power-of-two scale, in FP32 instructions
// only: v * scale is exact, so is its rounding to an integer r (|r| < 2^62),
// and |r| = hi 2^32 + lo with hi = floor(|r| 2^-32) and lo = |r| - hi 2^32 in
// [0, 2^32) is split exactly (lo's bits are a subset of |r|'s); the sign is
// applied to the 64-bit integer.  The result equals to_fixed((double)v, scale).
__device__ __forceinline__ long long to_fixed_f(float v, float scale, uint32_t* err) {
    const float s = v * scale;
    if (!(fabsf(s) < 4.6116860184273879e18f)) {   // 2^62
        raise_error(err, (v == v && fabsf(v) <= 3.4028234663852886e38f) ? GBR_ERR_OVERFLOW
                                                                         : GBR_ERR_NONFINITE);
        return 0;
    }
    const float r = __builtin_rintf(s);
    const float a = fabsf(r);
    const float hi = floorf(a * 2.3283064365386963e-10f);         // 2^-32
    const float lo = __builtin_fmaf(hi, -4294967296.0f, a);
    const unsigned long long u = ((unsigned long long)(uint32_t)hi << 32) | (uint32_t)lo;
    return r < 0.0f ? -(long long)u : (long long)u;
}

__device__ __forceinline__ void atomic_add_fx(int64_t* p, long long v) {
    if (v != 0)
        __hip_atomic_fetch_add(reinterpret_cast<unsigned long long*>(p),
                               static_cast<unsigned long long>(v), __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ double from_fixed(int64_t v, double inv_scale) {
    return (double)v * inv_scale;
}

// -------------------------------------------------------- wave reductions
// Index of the calling wavefront inside its workgroup, as a wave-uniform
// value: loads indexed by it (work items, replica offsets) become scalar loads.
__device__ __forceinline__ int wave_in_group() {
    return __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
}

// Sum of a 64-bit integer over the wavefront, in lane 63 (other lanes hold
// partial sums): an inclusive scan within each row of 16 lanes (DPP row_shr
// 1, 2, 4, 8), then the row totals carried up (row_bcast 15, 31).  Integer
// sums do not depend on order.
template <int CTRL, int ROWS>
__device__ __forceinline__ unsigned long long dpp_u64(unsigned long long v) {
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)v, CTRL, ROWS, 0xF, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)(v >> 32), CTRL, ROWS, 0xF, true);
    return ((unsigned long long)(uint32_t)hi << 32) | (uint32_t)lo;
}
__device__ __forceinline__ long long wave_sum_i64_lane63(long long x) {
    unsigned long long v = (unsigned long long)x;
    v += dpp_u64<0x111, 0xF>(v);   // row_shr:1
    v += dpp_u64<0x112, 0xF>(v);   // row_shr:2
    v += dpp_u64<0x114, 0xF>(v);   // row_shr:4
    v += dpp_u64<0x118, 0xF>(v);   // row_shr:8
    v += dpp_u64<0x142, 0xA>(v);   // row_bcast:15 into rows 1 and 3
    v += dpp_u64<0x143, 0xC>(v);   // row_bcast:31 into rows 2 and 3
    return (long long)v;
}

__device__ __forceinline__ double wave_sum_d(double v) {
    // doubles: butterfly through shuffles (used only once per tile)
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, GBR_WAVE);
    return v;
}

// Per-tile kernels sum per-replica values wavefront by wavefront (one tile
// each); this merges the wavefronts of one workgroup: every run of
// consecutive wavefronts of one replica (rep; rep < 0: nothing) is added into
// the run's first wavefront, whose lane 0 returns true with the run's totals
// in v, so that one large replica's tiles do not all meet at its slots in
// memory.  Every thread of the workgroup calls it (at most 16 wavefronts).
constexpr int MAX_GROUP_WAVES = 16;
template <int NV>
__device__ __forceinline__ bool group_runs_by_replica(int rep, long long (&v)[NV]) {
    __shared__ int s_rep[MAX_GROUP_WAVES];
    __shared__ long long s_v[NV][MAX_GROUP_WAVES];
    const int w = (int)(threadIdx.x >> 6), nw = (int)(blockDim.x >> 6), lane = threadIdx.x & 63;
    if (lane == 0) {
        s_rep[w] = rep;
        for (int k = 0; k < NV; ++k) s_v[k][w] = v[k];
    }
    __syncthreads();
    if (lane != 0 || rep < 0 || (w > 0 && s_rep[w - 1] == rep)) return false;
    for (int u = w + 1; u < nw && s_rep[u] == rep; ++u)
        for (int k = 0; k < NV; ++k) v[k] += s_v[k][u];
    return true;
}

// -------------------------------------------------- Philox4x32-10 (SC'11)
struct U4 { uint32_t x, y, z, w; };

__device__ __forceinline__ U4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                     uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
        uint32_t lo0 = 0xD2511F53u * c0, hi0 = __umulhi(0xD2511F53u, c0);
        uint32_t lo1 = 0xCD9E8D57u * c2, hi1 = __umulhi(0xCD9E8D57u, c2);
        uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
    }
    return {c0, c1, c2, c3};
}

// draw for (sub, entity, step, stream) keyed by seed
__device__ __forceinline__ U4 draw(uint64_t seed, uint32_t sub, uint32_t entity, uint64_t step,
                                   uint32_t stream) {
    return philox(sub, entity, (uint32_t)step,
                  (stream << 24) | (uint32_t)((step >> 32) & 0xFFFFFFu),
                  (uint32_t)seed, (uint32_t)(seed >> 32));
}

__device__ __forceinline__ double uniform53(uint32_t a, uint32_t b) {
    return ((double)(a >> 5) * 67108864.0 + (double)(b >> 6)) * (1.0 / 9007199254740992.0);
}

__device__ __forceinline__ uint32_t choose(uint32_t w, uint32_t n) {
    return (uint32_t)(((uint64_t)w * (uint64_t)n) >> 32);
}

__device__ __forceinline__ void normal2(U4 w, double& n0, double& n1) {
    double u1 = uniform53(w.x, w.y), u2 = uniform53(w.z, w.w);
    double rad = sqrt(-2.0 * log(1.0 - u1));
    double sn, cs;
    sincospi(2.0 * u2, &sn, &cs);
    n0 = rad * cs;
    n1 = rad * sn;
}

// ---------------------------------------------- descreening term (FP32)
// h(r; rt, s) for a sphere of radius s at distance r from an atom of offset
// radius rt: twice the integral over shells t >= rt of (covered fraction)/t^2.
//  - sphere inside the atom (r + s <= rt): 0
//  - distant sphere (r - s >= rt, s/r <= HCT_FAR_XMAX): (x^3/r) G(x^2), x = s/r
//    (evaluated in the pair kernels)
//  - otherwise the closed form with L = max(rt, |r - s|), U = r + s, plus the
//    engulfing term when rt < s - r (hct_closed).
__device__ __forceinline__ float poly_G(float y) {
    float p = hct_G_coef[HCT_G_DEG];
#pragma unroll
    for (int k = HCT_G_DEG - 1; k >= 0; --k) p = __builtin_fmaf(p, y, hct_G_coef[k]);
    return p;
}
__device__ __forceinline__ float poly_Q(float y) {
    float p = hct_Q_coef[HCT_Q_DEG];
#pragma unroll
    for (int k = HCT_Q_DEG - 1; k >= 0; --k) p = __builtin_fmaf(p, y, hct_Q_coef[k]);
    return p;
}

__device__ __forceinline__ float frcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float frsq(float x) { return __builtin_amdgcn_rsqf(x); }
// natural log through the hardware log2
__device__ __forceinline__ float flog(float x) { return __builtin_amdgcn_logf(x) * 0.69314718055994531f; }
__device__ __forceinline__ float fexp_neg(float x) { return __builtin_amdgcn_exp2f(-x * 1.4426950408889634f); }

__device__ __forceinline__ float hct_closed(float r, float rinv, float rt, float s) {
    float U = r + s;
    float rms = r - s;
    float L = fmaxf(rt, fabsf(rms));
    float iL = frcp(L), iU = frcp(U);
    float h = (iL - iU) + (iU * iU - iL * iL) * ((r * r - s * s) * 0.25f * rinv)
            + 0.5f * rinv * flog(L * iU);
    // engulfed: + 2 (1/rt - 1/L), written with one reciprocal of the pair's rt L
    if (rt < -rms) h += 2.0f * (L - rt) * frcp(rt * L);
    return h;
}

// dh/dr.  Distant sphere: -(x^3/r^2) Q(x^2) (in the pair kernels).  Otherwise
//   dh/dr = [ (r^2 + s^2)(1/U^2 - 1/L^2)/2 + ln(U/L) ] / (2 r^2)
// (the boundary terms of the shell integral vanish or cancel in every branch).
__device__ __forceinline__ float hct_dr_closed(float r, float rinv, float rt, float s) {
    float U = r + s;
    float L = fmaxf(rt, fabsf(r - s));
    float iL = frcp(L), iU = frcp(U);
    float a = (r * r + s * s) * (iU * iU - iL * iL) * 0.5f - flog(L * iU);
    return a * 0.5f * rinv * rinv;
}

// All three partials (for the radius adjoint).
//   dh/drt: overlap (L = rt): ((r - rt)^2 - s^2) / (2 r rt^3); engulfed: -2/rt^2; else 0
//   dh/ds : (s / (2r)) (1/L^2 - 1/U^2); distant sphere: 2 s^2 / (r^2 - s^2)^2
__device__ __forceinline__ void hct_grad3(float r, float rinv, float rt, float s,
                                          float& d_r, float& d_rt, float& d_s) {
    float x = s * rinv;
    float y = x * x;
    bool far = (r - s >= rt) && (x <= HCT_FAR_XMAX);
    if (far) {
        d_r = -(x * y * rinv * rinv) * poly_Q(y);
        d_rt = 0.0f;
        float lu = (r - s) * (r + s);
        float ilu = frcp(lu);
        d_s = 2.0f * s * s * ilu * ilu;
    } else if (r + s <= rt) {
        d_r = 0.0f; d_rt = 0.0f; d_s = 0.0f;
    } else {
        float U = r + s;
        float rms = r - s;
        bool at_rt = rt >= fabsf(rms);
        float L = at_rt ? rt : fabsf(rms);
        float iL = frcp(L), iU = frcp(U);
        float dd = iL * iL - iU * iU;
        d_r = ((r * r + s * s) * (-dd) * 0.5f - flog(L * iU)) * 0.5f * rinv * rinv;
        d_s = 0.5f * s * rinv * dd;
        float irt = frcp(rt);
        if (at_rt) {
            float t = r - rt;
            d_rt = (t * t - s * s) * 0.5f * rinv * irt * irt * irt;
        } else if (rt < -rms) {
            d_rt = -2.0f * irt * irt;
        } else {
            d_rt = 0.0f;
        }
    }
}

}  // namespace gbr
