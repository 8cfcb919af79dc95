// pair_kernels.hip -- the three O(N^2) pair passes of a GB evaluation.
//
// Work decomposition (same for the three passes).  Replica r with n atoms is
// cut into 64-atom J tiles and (64 * NI)-atom I blocks.  A work item
// (r, IB, J) is the set of pairs (i, j) with i in block IB, j in tile J and
// i < j (local indices), so every unordered pair of every replica belongs to
// exactly one item; items exist for J >= IB * NI.  One wavefront processes one
// item: lane l holds the NI atoms i = IB*64*NI + u*64 + l (u < NI) in
// registers and one atom of the J tile; the J atoms are broadcast one at a time
// through readlane (scalar registers).  Contributions to i accumulate per lane
// in FP32; contributions to the broadcast j are summed over the lane's NI
// atoms and then over the wavefront with DPP, and land in the lane that owns
// j.  At the end of the item every per-atom partial is rounded to 64-bit fixed
// point and added with an integer atomic, so the result does not depend on the
// order in which items run.  Invalid pairs (i >= j, or an I lane past the end
// of the replica) are removed with selects, never with dummy parameters.
//
// Items are visited grid-stride by a persistent grid whose block index is
// remapped so that the blocks of one XCD (blocks are dealt round-robin to the
// eight XCDs) walk a contiguous range of the item list, i.e. of replicas.
#include "gbr_device.h"
#include "gbr_internal.h"

using namespace gbr;

namespace {

__device__ __forceinline__ int logical_wave() {
    const int nb = gridDim.x, b = blockIdx.x;
    const int lb = (nb & 7) ? b : ((b & 7) * (nb >> 3) + (b >> 3));
    return lb * (blockDim.x >> 6) + (threadIdx.x >> 6);
}

__device__ __forceinline__ float sel(bool c, float v) { return c ? v : 0.0f; }

// ------------------------------------------------------------- descreening
template <int NI>
__global__ __launch_bounds__(256) void k_born_pair(
    const int2* __restrict__ items, int n_items, const int32_t* __restrict__ atom_off, int ntot,
    const float* __restrict__ xyz, const float* __restrict__ rho,
    const float* __restrict__ screen, float offset, int64_t* __restrict__ psi_fx,
    uint32_t* __restrict__ err)
{
    const int lane = threadIdx.x & 63;
    const int stride = gridDim.x * (blockDim.x >> 6);
    for (int it = logical_wave(); it < n_items; it += stride) {
        const int2 wi = items[it];
        const int rep = wi.x, IB = wi.y >> 16, J = wi.y & 0xFFFF;
        const int a0 = atom_off[rep], n = atom_off[rep + 1] - a0;
        float xi[NI], yi[NI], zi[NI], rti[NI], si[NI], acc[NI];
        int li[NI];
#pragma unroll
        for (int u = 0; u < NI; ++u) {
            li[u] = IB * 64 * NI + u * 64 + lane;
            const int a = a0 + min(li[u], n - 1);
            xi[u] = xyz[a]; yi[u] = xyz[ntot + a]; zi[u] = xyz[2 * ntot + a];
            rti[u] = rho[a] - offset;
            si[u] = screen[a] * rti[u];
            acc[u] = 0.0f;
        }
        const int jbase = J * 64;
        const int lj = jbase + lane;
        const int ja = a0 + min(lj, n - 1);
        const float xj = xyz[ja], yj = xyz[ntot + ja], zj = xyz[2 * ntot + ja];
        const float rtj = rho[ja] - offset, sj = screen[ja] * rtj;
        float accj = 0.0f;
        const int nj = min(64, n - jbase);
        for (int k = 0; k < nj; ++k) {
            const float xk = bcast(xj, k), yk = bcast(yj, k), zk = bcast(zj, k);
            const float rtk = bcast(rtj, k), sk = bcast(sj, k);
            const int lk = jbase + k;
            float cj = 0.0f;
#pragma unroll
            for (int u = 0; u < NI; ++u) {
                const float dx = xk - xi[u], dy = yk - yi[u], dz = zk - zi[u];
                const float r2 = dx * dx + dy * dy + dz * dz;
                const bool valid = li[u] < lk;
                const float rinv = frsq(r2);
                const float r = r2 * rinv;
                const float hij = hct_h(r, rinv, rti[u], sk);
                const float hji = hct_h(r, rinv, rtk, si[u]);
                acc[u] += sel(valid, hij);
                cj += sel(valid, hji);
            }
            const float tot = wave_sum(cj);
            accj += (lane == k) ? tot : 0.0f;
        }
#pragma unroll
        for (int u = 0; u < NI; ++u)
            if (li[u] < n) atomic_add_fx(&psi_fx[a0 + li[u]], to_fixed(acc[u], FX_FORCE, err));
        if (lj < n) atomic_add_fx(&psi_fx[ja], to_fixed(accj, FX_FORCE, err));
    }
}

// ---------------------------------------------- energy and direct forces
// Per pair at fixed Born radii:
//   e_C  = (k_e/eps_in) q_i q_j / r
//   e_GB = -k_e tau q_i q_j / f,  f^2 = r^2 + R_i R_j exp(-D),  D = r^2 / (4 R_i R_j)
//   e_LJ = 4 eps_ij (s^12 - s^6),  s = sigma_ij / r
// (1/r) dE/dr = -(e_C + 6 e4 (2 s^12 - s^6)) / r^2 - e_GB (1 - exp(-D)/4) / f^2
// dE/dR_i = -e_GB exp(-D) (1 + D) R_j / (2 f^2)
// dE/dq_i = k_e (1/(eps_in r) - tau/f) q_j
template <int NI, bool GQ>
__global__ __launch_bounds__(256) void k_energy_pair(
    const int2* __restrict__ items, int n_items, const int32_t* __restrict__ atom_off, int ntot,
    const float* __restrict__ xyz, const float* __restrict__ q, const float* __restrict__ Rb,
    const float* __restrict__ sigma, const float* __restrict__ eps, float ke, float ke_in,
    float tau, int64_t* __restrict__ force_fx, int64_t* __restrict__ dEdR_fx,
    int64_t* __restrict__ energy_fx, int64_t* __restrict__ dEdq_fx, uint32_t* __restrict__ err)
{
    const int lane = threadIdx.x & 63;
    const int stride = gridDim.x * (blockDim.x >> 6);
    const float ketau = ke * tau;
    for (int it = logical_wave(); it < n_items; it += stride) {
        const int2 wi = items[it];
        const int rep = wi.x, IB = wi.y >> 16, J = wi.y & 0xFFFF;
        const int a0 = atom_off[rep], n = atom_off[rep + 1] - a0;
        float xi[NI], yi[NI], zi[NI], qi[NI], Ri[NI], iRi[NI], hsi[NI], sei[NI];
        float fxi[NI], fyi[NI], fzi[NI], dRi[NI], dqi[NI];
        int li[NI];
#pragma unroll
        for (int u = 0; u < NI; ++u) {
            li[u] = IB * 64 * NI + u * 64 + lane;
            const int a = a0 + min(li[u], n - 1);
            xi[u] = xyz[a]; yi[u] = xyz[ntot + a]; zi[u] = xyz[2 * ntot + a];
            qi[u] = q[a]; Ri[u] = Rb[a]; iRi[u] = 1.0f / Ri[u];
            hsi[u] = 0.5f * sigma[a]; sei[u] = 2.0f * sqrtf(eps[a]);
            fxi[u] = fyi[u] = fzi[u] = dRi[u] = dqi[u] = 0.0f;
        }
        const int jbase = J * 64;
        const int lj = jbase + lane;
        const int ja = a0 + min(lj, n - 1);
        const float xj = xyz[ja], yj = xyz[ntot + ja], zj = xyz[2 * ntot + ja];
        const float qj = q[ja], Rj = Rb[ja], iRj = 1.0f / Rj;
        const float hsj = 0.5f * sigma[ja], sej = 2.0f * sqrtf(eps[ja]);
        float fxj = 0.0f, fyj = 0.0f, fzj = 0.0f, dRj = 0.0f, dqj = 0.0f;
        float e_c = 0.0f, e_gb = 0.0f, e_lj = 0.0f;
        const int nj = min(64, n - jbase);
        for (int k = 0; k < nj; ++k) {
            const float xk = bcast(xj, k), yk = bcast(yj, k), zk = bcast(zj, k);
            const float qk = bcast(qj, k), Rk = bcast(Rj, k), iRk = bcast(iRj, k);
            const float hsk = bcast(hsj, k), sek = bcast(sej, k);
            const int lk = jbase + k;
            float cx = 0.0f, cy = 0.0f, cz = 0.0f, cR = 0.0f, cq = 0.0f;
#pragma unroll
            for (int u = 0; u < NI; ++u) {
                const float dx = xk - xi[u], dy = yk - yi[u], dz = zk - zi[u];
                const float r2 = dx * dx + dy * dy + dz * dz;
                const bool valid = li[u] < lk;
                const float rinv = frsq(r2);
                const float rinv2 = rinv * rinv;
                const float qq = qi[u] * qk;
                const float ec = ke_in * qq * rinv;
                const float D = 0.25f * r2 * (iRi[u] * iRk);
                const float ex = fexp_neg(D);
                const float f2 = __builtin_fmaf(Ri[u] * Rk, ex, r2);
                const float finv = frsq(f2);
                const float finv2 = finv * finv;
                const float egb = -ketau * qq * finv;
                const float sg = hsi[u] + hsk;
                const float s2 = sg * sg * rinv2;
                const float s6 = s2 * s2 * s2;
                const float s12 = s6 * s6;
                const float e4 = sei[u] * sek;
                const float elj = e4 * (s12 - s6);
                float fs = -(ec + 6.0f * e4 * (2.0f * s12 - s6)) * rinv2
                           - egb * finv2 * (1.0f - 0.25f * ex);
                float gR = -0.5f * egb * finv2 * ex * (1.0f + D);
                fs = sel(valid, fs);
                gR = sel(valid, gR);
                e_c += sel(valid, ec);
                e_gb += sel(valid, egb);
                e_lj += sel(valid, elj);
                const float fx = fs * dx, fy = fs * dy, fz = fs * dz;
                fxi[u] += fx; fyi[u] += fy; fzi[u] += fz;
                cx -= fx; cy -= fy; cz -= fz;
                dRi[u] += gR * Rk;
                cR += gR * Ri[u];
                if (GQ) {
                    const float w = sel(valid, ke_in * rinv - ketau * finv);
                    dqi[u] += w * qk;
                    cq += w * qi[u];
                }
            }
            const float tx = wave_sum(cx), ty = wave_sum(cy), tz = wave_sum(cz);
            const float tR = wave_sum(cR);
            const bool mine = lane == k;
            fxj += mine ? tx : 0.0f;
            fyj += mine ? ty : 0.0f;
            fzj += mine ? tz : 0.0f;
            dRj += mine ? tR : 0.0f;
            if (GQ) {
                const float tq = wave_sum(cq);
                dqj += mine ? tq : 0.0f;
            }
        }
#pragma unroll
        for (int u = 0; u < NI; ++u) {
            if (li[u] < n) {
                const int a = a0 + li[u];
                atomic_add_fx(&force_fx[a], to_fixed(fxi[u], FX_FORCE, err));
                atomic_add_fx(&force_fx[ntot + a], to_fixed(fyi[u], FX_FORCE, err));
                atomic_add_fx(&force_fx[2 * ntot + a], to_fixed(fzi[u], FX_FORCE, err));
                atomic_add_fx(&dEdR_fx[a], to_fixed(dRi[u], FX_FORCE, err));
                if (GQ) atomic_add_fx(&dEdq_fx[a], to_fixed(dqi[u], FX_FORCE, err));
            }
        }
        if (lj < n) {
            atomic_add_fx(&force_fx[ja], to_fixed(fxj, FX_FORCE, err));
            atomic_add_fx(&force_fx[ntot + ja], to_fixed(fyj, FX_FORCE, err));
            atomic_add_fx(&force_fx[2 * ntot + ja], to_fixed(fzj, FX_FORCE, err));
            atomic_add_fx(&dEdR_fx[ja], to_fixed(dRj, FX_FORCE, err));
            if (GQ) atomic_add_fx(&dEdq_fx[ja], to_fixed(dqj, FX_FORCE, err));
        }
        const double sgb = wave_sum_d((double)e_gb);
        const double sc = wave_sum_d((double)e_c);
        const double slj = wave_sum_d((double)e_lj);
        if (lane == 0) {
            atomic_add_fx(&energy_fx[4 * rep + 0], to_fixed(sgb, FX_ENERGY, err));
            atomic_add_fx(&energy_fx[4 * rep + 1], to_fixed(sc, FX_ENERGY, err));
            atomic_add_fx(&energy_fx[4 * rep + 2], to_fixed(slj, FX_ENERGY, err));
        }
    }
}

// ------------------------------------------------- chain rule through psi
// F_i += g (x_j - x_i)/r,  g = c_i dh(r; rt_i, s_j)/dr + c_j dh(r; rt_j, s_i)/dr,
// c = (dE/dR)(dR/dpsi)(rho~/2).  With RHO also the pair part of dE/drho:
//   i: c_i dh_ij/drt + S_i c_j dh_ji/ds,   j: c_j dh_ji/drt + S_j c_i dh_ij/ds.
template <int NI, bool RHO>
__global__ __launch_bounds__(256) void k_chain_pair(
    const int2* __restrict__ items, int n_items, const int32_t* __restrict__ atom_off, int ntot,
    const float* __restrict__ xyz, const float* __restrict__ rho,
    const float* __restrict__ screen, const float* __restrict__ cc, float offset,
    int64_t* __restrict__ force_fx, int64_t* __restrict__ dEdrho_fx, uint32_t* __restrict__ err)
{
    const int lane = threadIdx.x & 63;
    const int stride = gridDim.x * (blockDim.x >> 6);
    for (int it = logical_wave(); it < n_items; it += stride) {
        const int2 wi = items[it];
        const int rep = wi.x, IB = wi.y >> 16, J = wi.y & 0xFFFF;
        const int a0 = atom_off[rep], n = atom_off[rep + 1] - a0;
        float xi[NI], yi[NI], zi[NI], rti[NI], si[NI], ci[NI], Si[NI];
        float fxi[NI], fyi[NI], fzi[NI], dri[NI];
        int li[NI];
#pragma unroll
        for (int u = 0; u < NI; ++u) {
            li[u] = IB * 64 * NI + u * 64 + lane;
            const int a = a0 + min(li[u], n - 1);
            xi[u] = xyz[a]; yi[u] = xyz[ntot + a]; zi[u] = xyz[2 * ntot + a];
            rti[u] = rho[a] - offset;
            Si[u] = screen[a];
            si[u] = Si[u] * rti[u];
            ci[u] = cc[a];
            fxi[u] = fyi[u] = fzi[u] = dri[u] = 0.0f;
        }
        const int jbase = J * 64;
        const int lj = jbase + lane;
        const int ja = a0 + min(lj, n - 1);
        const float xj = xyz[ja], yj = xyz[ntot + ja], zj = xyz[2 * ntot + ja];
        const float rtj = rho[ja] - offset, Sj = screen[ja], sj = Sj * rtj, cjv = cc[ja];
        float fxj = 0.0f, fyj = 0.0f, fzj = 0.0f, drj = 0.0f;
        const int nj = min(64, n - jbase);
        for (int k = 0; k < nj; ++k) {
            const float xk = bcast(xj, k), yk = bcast(yj, k), zk = bcast(zj, k);
            const float rtk = bcast(rtj, k), sk = bcast(sj, k), ck = bcast(cjv, k);
            const float Sk = RHO ? bcast(Sj, k) : 0.0f;
            const int lk = jbase + k;
            float cx = 0.0f, cy = 0.0f, cz = 0.0f, cr = 0.0f;
#pragma unroll
            for (int u = 0; u < NI; ++u) {
                const float dx = xk - xi[u], dy = yk - yi[u], dz = zk - zi[u];
                const float r2 = dx * dx + dy * dy + dz * dz;
                const bool valid = li[u] < lk;
                const float rinv = frsq(r2);
                const float r = r2 * rinv;
                float g;
                if (RHO) {
                    float dr_ij, drt_ij, ds_ij, dr_ji, drt_ji, ds_ji;
                    hct_grad3(r, rinv, rti[u], sk, dr_ij, drt_ij, ds_ij);
                    hct_grad3(r, rinv, rtk, si[u], dr_ji, drt_ji, ds_ji);
                    g = ci[u] * dr_ij + ck * dr_ji;
                    dri[u] += sel(valid, ci[u] * drt_ij + Si[u] * ck * ds_ji);
                    cr += sel(valid, ck * drt_ji + Sk * ci[u] * ds_ij);
                } else {
                    g = ci[u] * hct_dr(r, rinv, rti[u], sk) + ck * hct_dr(r, rinv, rtk, si[u]);
                }
                const float fs = sel(valid, g * rinv);
                const float fx = fs * dx, fy = fs * dy, fz = fs * dz;
                fxi[u] += fx; fyi[u] += fy; fzi[u] += fz;
                cx -= fx; cy -= fy; cz -= fz;
            }
            const float tx = wave_sum(cx), ty = wave_sum(cy), tz = wave_sum(cz);
            const bool mine = lane == k;
            fxj += mine ? tx : 0.0f;
            fyj += mine ? ty : 0.0f;
            fzj += mine ? tz : 0.0f;
            if (RHO) {
                const float tr = wave_sum(cr);
                drj += mine ? tr : 0.0f;
            }
        }
#pragma unroll
        for (int u = 0; u < NI; ++u) {
            if (li[u] < n) {
                const int a = a0 + li[u];
                atomic_add_fx(&force_fx[a], to_fixed(fxi[u], FX_FORCE, err));
                atomic_add_fx(&force_fx[ntot + a], to_fixed(fyi[u], FX_FORCE, err));
                atomic_add_fx(&force_fx[2 * ntot + a], to_fixed(fzi[u], FX_FORCE, err));
                if (RHO) atomic_add_fx(&dEdrho_fx[a], to_fixed(dri[u], FX_FORCE, err));
            }
        }
        if (lj < n) {
            atomic_add_fx(&force_fx[ja], to_fixed(fxj, FX_FORCE, err));
            atomic_add_fx(&force_fx[ntot + ja], to_fixed(fyj, FX_FORCE, err));
            atomic_add_fx(&force_fx[2 * ntot + ja], to_fixed(fzj, FX_FORCE, err));
            if (RHO) atomic_add_fx(&dEdrho_fx[ja], to_fixed(drj, FX_FORCE, err));
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

hipError_t launch_born_pair(const gbr_ctx* c, const float* xyz, const float* rho,
                            const float* screen, hipStream_t s)
{
    const PairList& L = list_for(c, c->ni_born);
    if (L.n_items == 0) return hipSuccess;
    dim3 grid(grid_for(c, L.n_items)), block(64 * c->shape.waves_per_group);
    const float off = (float)c->prm.offset;
#define GBR_BORN(NI) hipLaunchKernelGGL(k_born_pair<NI>, grid, block, 0, s, L.items, L.n_items, \
        c->atom_off, c->n_atoms, xyz, rho, screen, off, c->psi_fx, c->err)
    switch (L.ni) {
        case 1: GBR_BORN(1); break;
        case 2: GBR_BORN(2); break;
        case 4: GBR_BORN(4); break;
        default: GBR_BORN(8); break;
    }
#undef GBR_BORN
    return hipGetLastError();
}

hipError_t launch_energy_pair(const gbr_ctx* c, const float* xyz, const float* q,
                              const float* R, const float* sigma, const float* eps,
                              int64_t* force_fx, int64_t* energy_fx, int64_t* dEdq_fx,
                              hipStream_t s)
{
    const PairList& L = list_for(c, c->ni_energy);
    if (L.n_items == 0) return hipSuccess;
    dim3 grid(grid_for(c, L.n_items)), block(64 * c->shape.waves_per_group);
    const GBConstH k = make_const(c->prm);
#define GBR_EN(NI, GQ) hipLaunchKernelGGL((k_energy_pair<NI, GQ>), grid, block, 0, s, L.items, \
        L.n_items, c->atom_off, c->n_atoms, xyz, q, R, sigma, eps, k.ke, k.ke_in, k.tau, force_fx, \
        c->dEdR_fx, energy_fx, dEdq_fx, c->err)
    const bool gq = dEdq_fx != nullptr;
    switch (L.ni) {
        case 1: if (gq) GBR_EN(1, true); else GBR_EN(1, false); break;
        case 2: if (gq) GBR_EN(2, true); else GBR_EN(2, false); break;
        case 4: if (gq) GBR_EN(4, true); else GBR_EN(4, false); break;
        default: if (gq) GBR_EN(8, true); else GBR_EN(8, false); break;
    }
#undef GBR_EN
    return hipGetLastError();
}

hipError_t launch_chain_pair(const gbr_ctx* c, const float* xyz, const float* rho,
                             const float* screen, int64_t* force_fx, int64_t* dEdrho_fx,
                             hipStream_t s)
{
    const PairList& L = list_for(c, c->ni_chain);
    if (L.n_items == 0) return hipSuccess;
    dim3 grid(grid_for(c, L.n_items)), block(64 * c->shape.waves_per_group);
    const float off = (float)c->prm.offset;
#define GBR_CH(NI, RH) hipLaunchKernelGGL((k_chain_pair<NI, RH>), grid, block, 0, s, L.items, \
        L.n_items, c->atom_off, c->n_atoms, xyz, rho, screen, c->chain_c, off, force_fx, \
        dEdrho_fx, c->err)
    const bool rh = dEdrho_fx != nullptr;
    switch (L.ni) {
        case 1: if (rh) GBR_CH(1, true); else GBR_CH(1, false); break;
        case 2: if (rh) GBR_CH(2, true); else GBR_CH(2, false); break;
        case 4: if (rh) GBR_CH(4, true); else GBR_CH(4, false); break;
        default: if (rh) GBR_CH(8, true); else GBR_CH(8, false); break;
    }
#undef GBR_CH
    return hipGetLastError();
}

}  // namespace gbr
