// issue_rate.hip -- VALU issue-rate microbenchmark for gfx950.
//
// Each wavefront runs a fixed block of VALU instructions many times over
// eight (or more) independent register chains, so that no instruction waits
// on the one before it; the wavefront's own shader-clock cycles (s_memtime)
// over the loop give its issue rate.  With W wavefronts on every SIMD
// (workgroups of 256 threads put one wavefront on each of a CU's four SIMDs;
// W workgroups per CU), the SIMD's rate is W x instructions / cycles, quoted
// per quad-cycle (the VALU issue unit): 1 = one wave64 instruction every four
// cycles, 2 = two instructions from different wavefronts issued together.
//
// Every instruction is written in inline asm so that its encoding is the one
// named (VOP2, VOP3 with a negated operand, an SGPR operand, a literal, a
// transcendental, a DPP rotation); no packed-FP32 instruction is used.  A
// register written by a transcendental or read through DPP is not touched
// again for at least seven instructions.  Results are written out so that
// nothing is dead.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <cstdio>
#include <vector>

namespace {

// instruction mixes: 16 instructions per block
enum Mix : int {
    MIX_FMAC = 0,      // v_fmac_f32 (VOP2)
    MIX_FMA_NEG,       // v_fma_f32 with a negated operand (VOP3)
    MIX_MUL_SGPR,      // v_mul_f32 with an SGPR operand (VOP2)
    MIX_FMAAK,         // v_fmaak_f32 (VOP2 with a 32-bit literal)
    MIX_EXP,           // v_exp_f32 (transcendental)
    MIX_RSQ,           // v_rsq_f32 (transcendental)
    MIX_DPP,           // v_add_f32_dpp wave_rol:1
    MIX_FMAC_EXP_3_1,  // 12 v_fmac + 4 v_exp
    MIX_FMAC_EXP_7_1,  // 14 v_fmac + 2 v_exp
    MIX_FMAC_DPP_3_1,  // 12 v_fmac + 4 dpp adds
    MIX_FMAC_VOP3_1_1, // 8 v_fmac + 8 VOP3 v_fma (negated operand)
    MIX_FMAC_SGPR_1_1, // 8 v_fmac + 8 v_mul with an SGPR operand
    MIX_FMAC_LDSADD_3_1, // 12 v_fmac + 4 ds_add_f32 (LDS pipe)
    MIX_FMAC_LDSRD_7_1,  // 14 v_fmac + 2 ds_read_b128 (LDS pipe)
    MIX_FMAC_ROWROR_3_1, // 12 v_fmac + 4 v_add_f32_dpp row_ror:1 (rotation inside 16-lane rows)
    MIX_FMAC_BPERM_3_1,  // 12 v_fmac + 4 ds_bpermute_b32 (LDS crossbar), one wait per 16
    MIX_COUNT
};

#define FMAC(a) asm volatile("v_fmac_f32 %0, %1, %2" : "+v"(a) : "v"(x), "v"(y))
#define FMAN(a) asm volatile("v_fma_f32 %0, -%1, %2, %0" : "+v"(a) : "v"(x), "v"(y))
#define MULS(a) asm volatile("v_mul_f32 %0, %1, %0" : "+v"(a) : "s"(sv))
#define FMAK(a) asm volatile("v_fmaak_f32 %0, %0, %1, 0x3f800000" : "+v"(a) : "v"(y))
#define EXPT(t) asm volatile("v_exp_f32 %0, %0" : "+v"(t))
#define RSQT(t) asm volatile("v_rsq_f32 %0, %0" : "+v"(t))
#define DPPA(a) asm volatile("v_add_f32_dpp %0, %0, %1 wave_rol:1 row_mask:0xf bank_mask:0xf" : "+v"(a) : "v"(x))
#define ROWR(a) asm volatile("v_add_f32_dpp %0, %0, %1 row_ror:1 row_mask:0xf bank_mask:0xf" : "+v"(a) : "v"(x))
#define BPRM(t) asm volatile("ds_bpermute_b32 %0, %1, %0" : "+v"(t) : "v"(pa) : "memory")
#define LDSA(o) asm volatile("ds_add_f32 %0, %1 offset:" #o : : "v"(la), "v"(x) : "memory")
#define LDSR(q, o) asm volatile("ds_read_b128 %0, %1 offset:" #o "\n\ts_waitcnt lgkmcnt(0)" : "=v"(q) : "v"(la) : "memory")

template <int MIX>
__device__ __forceinline__ void block16(float (&a)[8], float (&t)[8], float x, float y, float sv,
                                        unsigned la, float4& q, unsigned pa) {
    if constexpr (MIX == MIX_FMAC) {
        FMAC(a[0]); FMAC(a[1]); FMAC(a[2]); FMAC(a[3]); FMAC(a[4]); FMAC(a[5]); FMAC(a[6]); FMAC(a[7]);
        FMAC(a[0]); FMAC(a[1]); FMAC(a[2]); FMAC(a[3]); FMAC(a[4]); FMAC(a[5]); FMAC(a[6]); FMAC(a[7]);
    } else if constexpr (MIX == MIX_FMA_NEG) {
        FMAN(a[0]); FMAN(a[1]); FMAN(a[2]); FMAN(a[3]); FMAN(a[4]); FMAN(a[5]); FMAN(a[6]); FMAN(a[7]);
        FMAN(a[0]); FMAN(a[1]); FMAN(a[2]); FMAN(a[3]); FMAN(a[4]); FMAN(a[5]); FMAN(a[6]); FMAN(a[7]);
    } else if constexpr (MIX == MIX_MUL_SGPR) {
        MULS(a[0]); MULS(a[1]); MULS(a[2]); MULS(a[3]); MULS(a[4]); MULS(a[5]); MULS(a[6]); MULS(a[7]);
        MULS(a[0]); MULS(a[1]); MULS(a[2]); MULS(a[3]); MULS(a[4]); MULS(a[5]); MULS(a[6]); MULS(a[7]);
    } else if constexpr (MIX == MIX_FMAAK) {
        FMAK(a[0]); FMAK(a[1]); FMAK(a[2]); FMAK(a[3]); FMAK(a[4]); FMAK(a[5]); FMAK(a[6]); FMAK(a[7]);
        FMAK(a[0]); FMAK(a[1]); FMAK(a[2]); FMAK(a[3]); FMAK(a[4]); FMAK(a[5]); FMAK(a[6]); FMAK(a[7]);
    } else if constexpr (MIX == MIX_EXP) {
        EXPT(t[0]); EXPT(t[1]); EXPT(t[2]); EXPT(t[3]); EXPT(t[4]); EXPT(t[5]); EXPT(t[6]); EXPT(t[7]);
        EXPT(a[0]); EXPT(a[1]); EXPT(a[2]); EXPT(a[3]); EXPT(a[4]); EXPT(a[5]); EXPT(a[6]); EXPT(a[7]);
    } else if constexpr (MIX == MIX_RSQ) {
        RSQT(t[0]); RSQT(t[1]); RSQT(t[2]); RSQT(t[3]); RSQT(t[4]); RSQT(t[5]); RSQT(t[6]); RSQT(t[7]);
        RSQT(a[0]); RSQT(a[1]); RSQT(a[2]); RSQT(a[3]); RSQT(a[4]); RSQT(a[5]); RSQT(a[6]); RSQT(a[7]);
    } else if constexpr (MIX == MIX_DPP) {
        DPPA(a[0]); DPPA(a[1]); DPPA(a[2]); DPPA(a[3]); DPPA(a[4]); DPPA(a[5]); DPPA(a[6]); DPPA(a[7]);
        DPPA(t[0]); DPPA(t[1]); DPPA(t[2]); DPPA(t[3]); DPPA(t[4]); DPPA(t[5]); DPPA(t[6]); DPPA(t[7]);
    } else if constexpr (MIX == MIX_FMAC_EXP_3_1) {
        FMAC(a[0]); FMAC(a[1]); FMAC(a[2]); EXPT(t[0]); FMAC(a[3]); FMAC(a[4]); FMAC(a[5]); EXPT(t[1]);
        FMAC(a[6]); FMAC(a[7]); FMAC(a[0]); EXPT(t[2]); FMAC(a[1]); FMAC(a[2]); FMAC(a[3]); EXPT(t[3]);
    } else if constexpr (MIX == MIX_FMAC_EXP_7_1) {
        FMAC(a[0]); FMAC(a[1]); FMAC(a[2]); FMAC(a[3]); FMAC(a[4]); FMAC(a[5]); FMAC(a[6]); EXPT(t[0]);
        FMAC(a[7]); FMAC(a[0]); FMAC(a[1]); FMAC(a[2]); FMAC(a[3]); FMAC(a[4]); FMAC(a[5]); EXPT(t[1]);
    } else if constexpr (MIX == MIX_FMAC_DPP_3_1) {
        FMAC(a[0]); FMAC(a[1]); FMAC(a[2]); DPPA(t[0]); FMAC(a[3]); FMAC(a[4]); FMAC(a[5]); DPPA(t[1]);
        FMAC(a[6]); FMAC(a[7]); FMAC(a[0]); DPPA(t[2]); FMAC(a[1]); FMAC(a[2]); FMAC(a[3]); DPPA(t[3]);
    } else if constexpr (MIX == MIX_FMAC_VOP3_1_1) {
        FMAC(a[0]); FMAN(t[0]); FMAC(a[1]); FMAN(t[1]); FMAC(a[2]); FMAN(t[2]); FMAC(a[3]); FMAN(t[3]);
        FMAC(a[4]); FMAN(t[4]); FMAC(a[5]); FMAN(t[5]); FMAC(a[6]); FMAN(t[6]); FMAC(a[7]); FMAN(t[7]);
    } else if constexpr (MIX == MIX_FMAC_SGPR_1_1) {
        FMAC(a[0]); MULS(t[0]); FMAC(a[1]); MULS(t[1]); FMAC(a[2]); MULS(t[2]); FMAC(a[3]); MULS(t[3]);
        FMAC(a[4]); MULS(t[4]); FMAC(a[5]); MULS(t[5]); FMAC(a[6]); MULS(t[6]); FMAC(a[7]); MULS(t[7]);
    } else if constexpr (MIX == MIX_FMAC_LDSADD_3_1) {
        FMAC(a[0]); FMAC(a[1]); FMAC(a[2]); LDSA(0); FMAC(a[3]); FMAC(a[4]); FMAC(a[5]); LDSA(256);
        FMAC(a[6]); FMAC(a[7]); FMAC(a[0]); LDSA(512); FMAC(a[1]); FMAC(a[2]); FMAC(a[3]); LDSA(768);
    } else if constexpr (MIX == MIX_FMAC_ROWROR_3_1) {
        FMAC(a[0]); FMAC(a[1]); FMAC(a[2]); ROWR(t[0]); FMAC(a[3]); FMAC(a[4]); FMAC(a[5]); ROWR(t[1]);
        FMAC(a[6]); FMAC(a[7]); FMAC(a[0]); ROWR(t[2]); FMAC(a[1]); FMAC(a[2]); FMAC(a[3]); ROWR(t[3]);
    } else if constexpr (MIX == MIX_FMAC_BPERM_3_1) {
        FMAC(a[0]); FMAC(a[1]); FMAC(a[2]); BPRM(t[0]); FMAC(a[3]); FMAC(a[4]); FMAC(a[5]); BPRM(t[1]);
        FMAC(a[6]); FMAC(a[7]); FMAC(a[0]); BPRM(t[2]); FMAC(a[1]); FMAC(a[2]); FMAC(a[3]); BPRM(t[3]);
        asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
    } else {
        // the wait after each read is the worst case: every read's latency exposed to the wavefront
        FMAC(a[0]); FMAC(a[1]); FMAC(a[2]); FMAC(a[3]); FMAC(a[4]); FMAC(a[5]); FMAC(a[6]); LDSR(q, 0);
        FMAC(a[7]); FMAC(a[0]); FMAC(a[1]); FMAC(a[2]); FMAC(a[3]); FMAC(a[4]); FMAC(a[5]); LDSR(q, 1024);
    }
}

// out[thread] keeps the registers live; cyc[wave] = {shader cycles, 100 MHz ticks}.
template <int MIX>
__global__ __launch_bounds__(256) void k_issue(float* __restrict__ out, uint64_t* __restrict__ cyc,
                                               int iters, float sv) {
    // per wavefront: 4 x 256 B of LDS for the add mix, 2 KB for the read mix
    __shared__ float lds[4][512];
    const int gid = blockIdx.x * blockDim.x + threadIdx.x;
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const float x = 1.0f + 1e-7f * (float)lane, y = 0.999f;
    for (int k = lane; k < 512; k += 64) lds[wv][k] = 0.0f;
    const unsigned la = (unsigned)(uintptr_t)&lds[wv][0] + 4u * lane
                      + (MIX == MIX_FMAC_LDSRD_7_1 ? 12u * lane : 0u);   // read mix: 16 B per lane
    float4 q = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    const unsigned pa = 4u * ((lane + 1) & 63);          // bpermute: read lane + 1 (a rotation)
    float a[8], t[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        a[k] = 0.5f + 0.01f * k;
        t[k] = 1.5f + 0.01f * k;
    }
    __syncthreads();
    const uint64_t c0 = __builtin_amdgcn_s_memtime(), r0 = __builtin_amdgcn_s_memrealtime();
    for (int i = 0; i < iters; ++i) {
        block16<MIX>(a, t, x, y, sv, la, q, pa);
        block16<MIX>(a, t, x, y, sv, la, q, pa);
        block16<MIX>(a, t, x, y, sv, la, q, pa);
        block16<MIX>(a, t, x, y, sv, la, q, pa);
    }
    const uint64_t c1 = __builtin_amdgcn_s_memtime(), r1 = __builtin_amdgcn_s_memrealtime();
    __syncthreads();
    float s = q.x + q.y + q.z + q.w + lds[wv][lane];
#pragma unroll
    for (int k = 0; k < 8; ++k) s += a[k] + t[k];
    out[gid] = s;
    if ((threadIdx.x & 63) == 0) {
        const int w = gid >> 6;
        cyc[2 * w] = c1 - c0;
        cyc[2 * w + 1] = r1 - r0;
    }
}

template <int MIX>
hipError_t launch(int grid, float* out, uint64_t* cyc, int iters, float sv) {
    hipLaunchKernelGGL(k_issue<MIX>, dim3(grid), dim3(256), 0, 0, out, cyc, iters, sv);
    return hipGetLastError();
}

typedef hipError_t (*Launcher)(int, float*, uint64_t*, int, float);
const Launcher kLaunch[MIX_COUNT] = {
    launch<0>, launch<1>, launch<2>, launch<3>, launch<4>, launch<5>,
    launch<6>, launch<7>, launch<8>, launch<9>, launch<10>, launch<11>, launch<12>, launch<13>,
    launch<14>, launch<15>};

}  // namespace

extern "C" {

// Runs mix `mix` with `waves_per_simd` workgroups of 256 threads per CU for
// `iters` x 64 instructions per wavefront.  Outputs: ipq (wave64
// instructions per quad-cycle per SIMD over the kernel's event-timed
// duration at the measured clock), mhz (shader clock: s_memtime cycles over
// s_memrealtime's 100 MHz ticks, median wavefront), and the milliseconds.
// Returns 0 or a HIP error code.
int issue_rate_run(int mix, int waves_per_simd, int iters, double* ipq, double* mhz, double* ms) {
    if (mix < 0 || mix >= MIX_COUNT || waves_per_simd < 1 || waves_per_simd > 8 || iters < 1) return -1;
    int dev = 0, n_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess) return -2;
    if (hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return -2;
    const int grid = n_cu * waves_per_simd;
    const int waves = grid * 4;
    float* out = nullptr;
    uint64_t* cyc = nullptr;
    hipEvent_t e0, e1;
    if (hipMalloc(&out, sizeof(float) * (size_t)grid * 256) != hipSuccess) return -3;
    if (hipMalloc(&cyc, sizeof(uint64_t) * 2 * (size_t)waves) != hipSuccess) return -3;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    hipError_t e = kLaunch[mix](grid, out, cyc, 4, 1.0001f);     // warm-up
    if (e == hipSuccess) e = hipDeviceSynchronize();
    (void)hipEventRecord(e0, 0);
    if (e == hipSuccess) e = kLaunch[mix](grid, out, cyc, iters, 1.0001f);
    (void)hipEventRecord(e1, 0);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    std::vector<uint64_t> h(2 * (size_t)waves);
    if (e == hipSuccess) e = hipMemcpy(h.data(), cyc, h.size() * sizeof(uint64_t), hipMemcpyDeviceToHost);
    float t = 0.0f;
    (void)hipEventElapsedTime(&t, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipFree(out);
    (void)hipFree(cyc);
    if (e != hipSuccess) return (int)e;
    std::vector<uint64_t> c(waves), r(waves);
    for (int w = 0; w < waves; ++w) { c[w] = h[2 * w]; r[w] = h[2 * w + 1]; }
    std::sort(c.begin(), c.end());
    std::sort(r.begin(), r.end());
    const double cyc_med = (double)c[waves / 2], rt_med = (double)r[waves / 2];
    const double instr = 64.0 * iters * waves;          // wave instructions in the timed launch
    *mhz = cyc_med / (rt_med / 100.0);                  // s_memrealtime ticks at 100 MHz
    *ipq = instr * 4.0 / ((double)t * 1e-3 * (*mhz) * 1e6 * (4.0 * n_cu));
    *ms = t;
    return 0;
}

int issue_rate_mix_count(void) { return MIX_COUNT; }

}  // extern "C"
