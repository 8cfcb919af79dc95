// atom_kernels.hip -- O(N) per-atom stages of a GB evaluation: the OBC
// rescaling of the descreening sums, the chain coefficients with the GB self
// terms, the radius adjoint's per-atom part, fixed-point conversion.
//
// Kernels that reduce into per-replica totals run one wavefront per 64-atom
// tile (the tile list carries the replica), reduce in FP64 across the wave and
// add one fixed-point value per tile; the others are flat over atoms.
#include "gbr_device.h"
#include "gbr_internal.h"

using namespace gbr;

namespace {

__global__ void k_zero_i64(int64_t* __restrict__ p, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

// psi_i = rho~_i * (1/2) sum_j h_ij;  1/R = 1/rho~ - tanh(alpha psi - beta psi^2 + gamma psi^3)/rho
__device__ __forceinline__ void born_rescale(int a, const float* __restrict__ rho,
                                             const int64_t* __restrict__ psi_fx, double offset,
                                             double alpha, double beta, double gamma,
                                             float* __restrict__ R, float* __restrict__ dRdpsi,
                                             double* __restrict__ psi_out, uint32_t* __restrict__ err)
{
    const double rh = rho[a], rt = rh - offset;
    const double ps = rt * 0.5 * from_fixed(psi_fx[a], INV_FX_FORCE);
    const double phi = ps * (alpha + ps * (-beta + ps * gamma));
    const double th = tanh(phi);
    const double invR = 1.0 / rt - th / rh;
    double Rv = 1.0 / invR;
    if (!(invR > 0.0) || !(Rv < 1.0e30)) {
        raise_error(err, GBR_ERR_RADIUS);
        Rv = rt;
    }
    R[a] = (float)Rv;
    dRdpsi[a] = (float)(Rv * Rv * (1.0 - th * th) * (alpha - 2.0 * beta * ps + 3.0 * gamma * ps * ps) / rh);
    if (psi_out) psi_out[a] = ps;
}

__global__ __launch_bounds__(256) void k_born_finalize(
    const int2* __restrict__ tiles, int n_tiles, const int32_t* __restrict__ atom_off,
    const float* __restrict__ rho, const int64_t* __restrict__ psi_fx, double offset,
    double alpha, double beta, double gamma, float* __restrict__ R, float* __restrict__ dRdpsi,
    double* __restrict__ psi_out, uint32_t* __restrict__ err)
{
    const int t = blockIdx.x * (blockDim.x >> 6) + wave_in_group();
    if (t >= n_tiles) return;
    const int lane = threadIdx.x & 63;
    const int2 tl = tiles[t];
    const int a0 = atom_off[tl.x], n = atom_off[tl.x + 1] - a0;
    const int li = tl.y * 64 + lane;
    if (li >= n) return;
    born_rescale(a0 + li, rho, psi_fx, offset, alpha, beta, gamma, R, dRdpsi, psi_out, err);
}

// The same over a flat range of atoms (no tile list); thread 0 also checks
// that the replicas end at n atoms.
__global__ __launch_bounds__(256) void k_born_finalize_flat(
    int n, int n_rep, const int32_t* __restrict__ atom_off, const float* __restrict__ rho,
    const int64_t* __restrict__ psi_fx, double offset, double alpha, double beta, double gamma,
    float* __restrict__ R, float* __restrict__ dRdpsi, double* __restrict__ psi_out,
    uint32_t* __restrict__ err)
{
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a == 0 && atom_off[n_rep] != n) raise_error(err, GBR_ERR_LAYOUT);
    if (a < n) born_rescale(a, rho, psi_fx, offset, alpha, beta, gamma, R, dRdpsi, psi_out, err);
}

// With kg(R) = k_e g(R) = (k_e tau + (k_e/eps_out)(1 - exp(-kappa R))) / R (tau/R
// without salt): dE/dR_i = pair part - (1/2) q_i^2 kg'(R_i);
// c_i = dE/dR_i * dR_i/dpsi_i * rho~_i/2; E_GB self = -(1/2) q_i^2 kg(R_i) added
// to the replica's energy; dE/dq_i self = -q_i kg(R_i).
__global__ __launch_bounds__(512) void k_coef(
    const int2* __restrict__ tiles, int n_tiles, const int32_t* __restrict__ atom_off,
    const float* __restrict__ q, const float* __restrict__ rho, const float* __restrict__ R,
    const float* __restrict__ dRdpsi, const int64_t* __restrict__ dEdR_fx, double ketau,
    double keout, double kappa, double offset, double* __restrict__ dEdR, float* __restrict__ cc,
    int64_t* __restrict__ energy_fx, int64_t* __restrict__ dEdq_fx, int64_t* __restrict__ e_stripe,
    uint64_t* __restrict__ step, uint32_t* __restrict__ err)
{
    const int t = blockIdx.x * (blockDim.x >> 6) + wave_in_group();
    const int lane = threadIdx.x & 63;
    // inside md_step: the step counter advances here, once per step (nothing in
    // this kernel reads it; the next step's kernels and the exchange do)
    if (step && t == 0 && lane == 0) step[0] = step[0] + 1;
    int rep = -1;
    long long v[1] = {0};
    if (t < n_tiles) {
        const int2 tl = tiles[t];
        const int a0 = atom_off[tl.x], n = atom_off[tl.x + 1] - a0;
        const int li = tl.y * 64 + lane;
        double eself = 0.0;
        if (li < n) {
            const int a = a0 + li;
            const double qa = q[a], Ra = R[a];
            double kg = ketau / Ra, dkg = -ketau / (Ra * Ra);
            if (kappa > 0.0) {
                const double es = exp(-kappa * Ra);
                kg = (ketau + keout * (1.0 - es)) / Ra;
                dkg = -kg / Ra + keout * kappa * es / Ra;
            }
            const double g = from_fixed(dEdR_fx[a], INV_FX_FORCE) - 0.5 * qa * qa * dkg;
            dEdR[a] = g;
            cc[a] = (float)(g * (double)dRdpsi[a] * 0.5 * ((double)rho[a] - offset));
            eself = -0.5 * qa * qa * kg;
            if (dEdq_fx) dEdq_fx[a] += to_fixed(-qa * kg, FX_FORCE, err);
        }
        rep = tl.x;
        v[0] = to_fixed(wave_sum_d(eself), FX_ENERGY, err);
    }
    if (group_runs_by_replica<1>(rep, v)) atomic_add_fx(&energy_fx[4 * rep], v[0]);
    // the replica's first tile also folds the energy pass's stripes into its
    // three energy slots and clears them for the next evaluation
    if (t < n_tiles && tiles[t].y == 0) {
        long long e[3] = {0, 0, 0};
        if (lane < E_STRIPES) {
            int64_t* d = e_stripe + ((size_t)rep * E_STRIPES + lane) * E_STRIPE_LEN;
            for (int k = 0; k < 3; ++k) { e[k] = d[k]; d[k] = 0; }
        }
        for (int k = 0; k < 3; ++k)
            for (int off = E_STRIPES / 2; off > 0; off >>= 1) e[k] += __shfl_xor(e[k], off, GBR_WAVE);
        if (lane == 0)
            for (int k = 0; k < 3; ++k) atomic_add_fx(&energy_fx[4 * rep + k], e[k]);
    }
}

// per-atom part of dE/drho_i: dE/dR_i [R^2 (1/rho~^2 - tanh/rho^2) + dR/dpsi * psi/rho~]
__global__ void k_rho_finalize(int ntot, const float* __restrict__ rho,
                               const double* __restrict__ psi, const double* __restrict__ dEdR,
                               double offset, double alpha, double beta, double gamma,
                               int64_t* __restrict__ dEdrho_fx, uint32_t* __restrict__ err)
{
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= ntot) return;
    const double rh = rho[a], rt = rh - offset, ps = psi[a];
    const double phi = ps * (alpha + ps * (-beta + ps * gamma));
    const double th = tanh(phi);
    const double Rv = 1.0 / (1.0 / rt - th / rh);
    const double dRdp = Rv * Rv * (1.0 - th * th) * (alpha - 2.0 * beta * ps + 3.0 * gamma * ps * ps) / rh;
    const double fixed = Rv * Rv * (1.0 / (rt * rt) - th / (rh * rh));
    const double v = dEdR[a] * (fixed + dRdp * ps / rt);
    dEdrho_fx[a] += to_fixed(v, FX_FORCE, err);
}

__global__ void k_fx_to_float(int ntot, int n_rep, int comps, const int32_t* __restrict__ atom_off,
                              const int64_t* __restrict__ src, double inv, const double* __restrict__ scale,
                              double sign, float* __restrict__ dst)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= (int64_t)ntot * comps) return;
    double f = sign * (double)src[i] * inv;
    if (scale) {
        const int a = (int)(i % ntot);
        int lo = 0, hi = n_rep;   // replica of atom a: atom_off[lo] <= a < atom_off[lo+1]
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (atom_off[mid] <= a) lo = mid; else hi = mid;
        }
        f *= scale[lo];
    }
    dst[i] = (float)f;
}

__global__ void k_energies(int n_rep, const int64_t* __restrict__ e, double* __restrict__ out) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n_rep) return;
    double t = 0.0;
    for (int c = 0; c < 4; ++c) {
        const double v = from_fixed(e[4 * r + c], INV_FX_ENERGY);
        out[5 * r + c] = v;
        if (c < 3) t += v;
    }
    out[5 * r + 4] = t;
}

int tile_grid(const gbr_ctx* c) { return (c->n_tiles + 3) / 4; }

}  // namespace

namespace gbr {

GBConstH make_const(const gbr_gb_params& p) {
    GBConstH k;
    k.ke_d = p.k_e;
    k.ke_in_d = p.k_e / p.eps_in;
    k.tau_d = 1.0 / p.eps_in - 1.0 / p.eps_out;
    k.offset_d = p.offset;
    k.alpha = p.alpha; k.beta = p.beta; k.gamma = p.gamma;
    k.ke = (float)k.ke_d; k.ke_in = (float)k.ke_in_d; k.tau = (float)k.tau_d;
    k.offset = (float)p.offset;
    return k;
}

hipError_t launch_zero_i64(int64_t* p, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(k_zero_i64, dim3((unsigned)blocks), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

hipError_t launch_born_finalize(const gbr_ctx* c, const float* rho, float* R, float* dRdpsi,
                                double* psi, hipStream_t s) {
    hipLaunchKernelGGL(k_born_finalize, dim3(tile_grid(c)), dim3(256), 0, s, c->tiles, c->n_tiles,
                       c->atom_off, rho, c->psi_fx, c->prm.offset, c->prm.alpha, c->prm.beta,
                       c->prm.gamma, R, dRdpsi, psi, c->err);
    return hipGetLastError();
}

hipError_t launch_born_finalize_flat(const gbr_gb_params& p, int n_atoms, int n_rep,
                                     const int32_t* atom_off, const float* rho, const int64_t* psi_fx,
                                     float* R, float* dRdpsi, double* psi, uint32_t* err, hipStream_t s) {
    hipLaunchKernelGGL(k_born_finalize_flat, dim3((n_atoms + 255) / 256), dim3(256), 0, s, n_atoms, n_rep,
                       atom_off, rho, psi_fx, p.offset, p.alpha, p.beta, p.gamma, R, dRdpsi, psi, err);
    return hipGetLastError();
}

hipError_t launch_coef(const gbr_ctx* c, const float* q, const float* rho, const float* R,
                       const float* dRdpsi, int64_t* energy_fx, int64_t* dEdq_fx, uint64_t* step,
                       hipStream_t s) {
    const GBConstH k = make_const(c->prm);
    hipLaunchKernelGGL(k_coef, dim3((c->n_tiles + 7) / 8), dim3(512), 0, s, c->tiles, c->n_tiles,
                       c->atom_off, q, rho, R, dRdpsi, c->dEdR_fx, k.ke_d * k.tau_d,
                       c->prm.k_e / c->prm.eps_out, c->prm.kappa, c->prm.offset,
                       c->dEdR, c->chain_c, energy_fx, dEdq_fx, c->e_stripe, step, c->err);
    return hipGetLastError();
}

hipError_t launch_rho_finalize(const gbr_ctx* c, const float* rho, const float* R,
                               const float* dRdpsi, const double* psi, int64_t* dEdrho_fx,
                               hipStream_t s) {
    (void)R; (void)dRdpsi;
    hipLaunchKernelGGL(k_rho_finalize, dim3((c->n_atoms + 255) / 256), dim3(256), 0, s,
                       c->n_atoms, rho, psi, c->dEdR, c->prm.offset, c->prm.alpha, c->prm.beta,
                       c->prm.gamma, dEdrho_fx, c->err);
    return hipGetLastError();
}

hipError_t launch_fx_to_float(const gbr_ctx* c, const int64_t* src, int comps, int bits,
                              const double* scale, int sign, float* dst, hipStream_t s) {
    const int64_t n = (int64_t)c->n_atoms * comps;
    hipLaunchKernelGGL(k_fx_to_float, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                       c->n_atoms, c->n_rep, comps, c->atom_off, src, ldexp(1.0, -bits), scale,
                       (double)sign, dst);
    return hipGetLastError();
}

hipError_t launch_energies(const gbr_ctx* c, const int64_t* e, double* out, hipStream_t s) {
    hipLaunchKernelGGL(k_energies, dim3((c->n_rep + 127) / 128), dim3(128), 0, s, c->n_rep, e, out);
    return hipGetLastError();
}

}  // namespace gbr
