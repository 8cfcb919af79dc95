// md_kernels.hip -- the cheap O(N) and O(R) parts of a C(pH,E)MD / REMD
// step that stay on the device: the BAOAB Langevin updates, the tether, the
// titration Monte Carlo attempts, and the replica-exchange attempts.
#include <cfloat>

#include "gbr_device.h"
#include "gbr_internal.h"

using namespace gbr;

namespace {

// ----------------------------------------------------------- step counter
// step[0] = index n of the step being executed; one thread of the step's
// k_coef (a kernel that does not read it, run once per step after the step's
// Langevin half and its Monte Carlo attempts) advances it to n + 1.
__global__ void k_set_step(uint64_t* step, uint64_t step0) { step[0] = step0; }

// Scale l of replica rep's GB + Coulomb + LJ energy (its Hamiltonian level).
__device__ __forceinline__ double ham_scale(const double* __restrict__ H_scale,
                                            const int32_t* __restrict__ target_idx, int rep) {
    return H_scale ? H_scale[target_idx[GBR_N_DIMS * rep + GBR_DIM_H]] : 1.0;
}

// A fixed-point force scaled by l (unchanged, bit for bit, at l = 1).
__device__ __forceinline__ int64_t scale_fx(int64_t f, double l, uint32_t* err) {
    return l == 1.0 ? f : to_fixed(l * from_fixed(f, INV_FX_FORCE), FX_FORCE, err);
}

// ------------------------------------------------------ B, A, O, A stages
// v += dt/2 F/m;  x += dt/2 v;  v = c1 v + c2 sqrt(kT/m) xi;  x += dt/2 v.
// Also clears the accumulators of the force evaluation that follows, after
// handing the previous step's kinetic energy to ke (may be NULL).
// MID: the kernel also closes the previous step (what k_md_last does, with
// the same roundings): the pair forces scaled by the replica's Hamiltonian
// scale, tether forces at the current positions, and the final half kick.  Used when nothing reads the previous step's end state (no
// exchange attempt after it, not the last step of the call), so that step's
// kinetic and tether energies are not formed; the kinetic-energy accumulator
// then stays at zero.
template <bool MID>
__global__ __launch_bounds__(256) void k_md_first(
    const int2* __restrict__ tiles, int n_tiles, const int32_t* __restrict__ atom_off, int ntot,
    const uint64_t* __restrict__ step, uint64_t seed, double hdt, double c1, double c2,
    const float* __restrict__ mass, const double* __restrict__ T_vals,
    const double* __restrict__ H_scale, const int32_t* __restrict__ target_idx,
    float* __restrict__ xyz, float* __restrict__ v,
    int64_t* __restrict__ force_fx, int64_t* __restrict__ energy_fx, int64_t* __restrict__ psi_fx,
    int64_t* __restrict__ dEdR_fx, int64_t* __restrict__ ke_fx, double* __restrict__ ke,
    const float* __restrict__ x0, double k_t, uint32_t* __restrict__ err)
{
    const int t = blockIdx.x * (blockDim.x >> 6) + wave_in_group();
    if (t >= n_tiles) return;
    const int lane = threadIdx.x & 63;
    const int2 tl = tiles[t];
    const int rep = tl.x;
    const int a0 = atom_off[rep], n = atom_off[rep + 1] - a0;
    const int li = tl.y * 64 + lane;
    if (tl.y == 0 && lane < 4) energy_fx[4 * rep + lane] = 0;
    if (!MID && tl.y == 0 && lane == 0) {
        if (ke) ke[rep] = from_fixed(ke_fx[rep], INV_FX_ENERGY);
        ke_fx[rep] = 0;
    }
    if (li >= n) return;
    const int a = a0 + li;
    const uint64_t nstep = step[0];
    const double kT = KB * T_vals[target_idx[GBR_N_DIMS * rep + GBR_DIM_T]];
    const double lam = MID ? ham_scale(H_scale, target_idx, rep) : 1.0;
    const double im = ACC_CONV / (double)mass[a];
    const double sd = sqrt(kT * im);
    double xi[4];
    normal2(draw(seed, 2u * li, (uint32_t)rep, nstep, STREAM_O), xi[0], xi[1]);
    normal2(draw(seed, 2u * li + 1u, (uint32_t)rep, nstep, STREAM_O), xi[2], xi[3]);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const int64_t idx = (int64_t)d * ntot + a;
        double vv = v[idx], xx = xyz[idx];
        int64_t f = force_fx[idx];
        if (MID) {
            const double dx = xx - (double)x0[idx];
            f = scale_fx(f, lam, err) + to_fixed(-2.0 * k_t * dx, FX_FORCE, err);
            vv = (double)(float)(vv + hdt * from_fixed(f, INV_FX_FORCE) * im);
        }
        vv += hdt * from_fixed(f, INV_FX_FORCE) * im;
        xx += hdt * vv;
        vv = c1 * vv + c2 * sd * xi[d];
        xx += hdt * vv;
        v[idx] = (float)vv;
        xyz[idx] = (float)xx;
        force_fx[idx] = 0;
    }
    psi_fx[a] = 0;
    dEdR_fx[a] = 0;
}

// The pair forces scaled by the replica's Hamiltonian scale, plus the tether
// k |x - x0|^2 (its energy in the replica's slot 3); then (kick) v += dt/2 F/m
// and the kinetic energy; one tile per wavefront, eight per workgroup.
__global__ __launch_bounds__(512) void k_md_last(
    const int2* __restrict__ tiles, int n_tiles, const int32_t* __restrict__ atom_off,
    int ntot, double hdt, double k_t, const double* __restrict__ H_scale,
    const int32_t* __restrict__ target_idx, const float* __restrict__ mass,
    const float* __restrict__ x0, const float* __restrict__ xyz, float* __restrict__ vel,
    int64_t* __restrict__ force_fx, int64_t* __restrict__ energy_fx, int64_t* __restrict__ ke_fx,
    int kick, uint32_t* __restrict__ err)
{
    const int t = blockIdx.x * (blockDim.x >> 6) + wave_in_group();
    const int lane = threadIdx.x & 63;
    int rep = -1;
    long long v[2] = {0, 0};
    if (t < n_tiles) {
        const int2 tl = tiles[t];
        rep = tl.x;
        const int a0 = atom_off[rep], n = atom_off[rep + 1] - a0;
        const int li = tl.y * 64 + lane;
        double et = 0.0, kin = 0.0;
        if (li < n) {
            const int a = a0 + li;
            const double m = mass[a], im = ACC_CONV / m;
            const double lam = ham_scale(H_scale, target_idx, rep);
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                const int64_t idx = (int64_t)d * ntot + a;
                const double dx = (double)xyz[idx] - (double)x0[idx];
                et += k_t * dx * dx;
                const int64_t f = scale_fx(force_fx[idx], lam, err) + to_fixed(-2.0 * k_t * dx, FX_FORCE, err);
                force_fx[idx] = f;
                double vv = vel[idx];
                if (kick) {
                    vv += hdt * from_fixed(f, INV_FX_FORCE) * im;
                    vel[idx] = (float)vv;
                }
                kin += 0.5 * m * (double)(float)vv * (double)(float)vv / ACC_CONV;
            }
        }
        v[0] = to_fixed(wave_sum_d(et), FX_ENERGY, err);
        v[1] = to_fixed(wave_sum_d(kin), FX_ENERGY, err);
    }
    if (group_runs_by_replica<2>(rep, v)) {
        atomic_add_fx(&energy_fx[4 * rep + 3], v[0]);
        atomic_add_fx(&ke_fx[rep], v[1]);
    }
}

__global__ void k_ke_out(int n_rep, const int64_t* __restrict__ ke_fx, double* __restrict__ ke) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r < n_rep) ke[r] = from_fixed(ke_fx[r], INV_FX_ENERGY);
}

// ------------------------------------------------------------ titration
// Electrostatic energy change of giving site `site` the charges of state
// `nw`, at fixed Born radii:
//   dE = sum_k d_k (K q)_k + 1/2 sum_{k,l} d_k d_l K_kl,   d = q_new - q on the site.
// The sum over the replica's atoms j in (K q)_k is split into chunks of
// TI_CHUNK atoms, one workgroup each (the quadratic term goes with chunk 0);
// the chunk sums meet in a 64-bit fixed-point accumulator (2^32 per kcal/mol),
// so the total does not depend on the order the workgroups finish in.
constexpr int MAX_SITE = 64;
constexpr int TB = 256;
constexpr int TI_CHUNK = 2048;

struct SiteSmem {
    float x[MAX_SITE], y[MAX_SITE], z[MAX_SITE], R[MAX_SITE], d[MAX_SITE], qn[MAX_SITE];
    int atom[MAX_SITE];
    double red[TB / 64];
};

__device__ double block_sum_d(double v, double* red) {
    v = wave_sum_d(v);
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[w] = v;
    __syncthreads();
    double s = 0.0;
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) s += red[i];
    return s;
}

// Salt and the pair cutoff in the titration kernel: keout = k_e / eps_out,
// kappa (1/A, 0: no salt), cut2 = cut^2 (FLT_MAX: no cutoff).
struct Screening {
    float keout, kappa, cut2;
};

// k_e g(f) of the GB term: (k_e tau + (k_e/eps_out)(1 - exp(-kappa f))) / f, given
// 1/f; k_e tau / f without salt.
__device__ __forceinline__ float kg_of(float finv, float ketau, const Screening& sc) {
    if (sc.kappa > 0.0f) {
        const float es = fexp_neg(sc.kappa / finv);
        return (ketau + sc.keout * (1.0f - es)) * finv;
    }
    return ketau * finv;
}

// The part of dE from atoms j0 .. j1-1 (plus the quadratic term if quad),
// summed over the workgroup; the result is valid in every thread.
__device__ double site_delta_e(SiteSmem& sm, int m, int j0, int j1, bool quad_term, int ntot,
                               const float* __restrict__ xyz, const float* __restrict__ q,
                               const float* __restrict__ R, float ke_in, float ketau, Screening sc)
{
    float lin = 0.0f;
    for (int j = j0 + (int)threadIdx.x; j < j1; j += blockDim.x) {
        const float xj = xyz[j], yj = xyz[ntot + j], zj = xyz[2 * ntot + j];
        const float qj = q[j], Rj = R[j];
        float acc = 0.0f;
        for (int k = 0; k < m; ++k) {
            float K;
            if (sm.atom[k] == j) {
                K = -kg_of(1.0f / Rj, ketau, sc);
            } else {
                const float dx = xj - sm.x[k], dy = yj - sm.y[k], dz = zj - sm.z[k];
                const float r2 = dx * dx + dy * dy + dz * dz;
                const float rinv = frsq(r2);
                const float ex = fexp_neg(0.25f * r2 / (sm.R[k] * Rj));
                const float finv = frsq(__builtin_fmaf(sm.R[k] * Rj, ex, r2));
                K = (r2 < sc.cut2) ? ke_in * rinv - kg_of(finv, ketau, sc) : 0.0f;
            }
            acc += sm.d[k] * K;
        }
        lin += acc * qj;
    }
    float quad = 0.0f;
    for (int t = threadIdx.x; quad_term && t < m * m; t += blockDim.x) {
        const int k = t / m, l = t % m;
        float K;
        if (k == l) {
            K = -kg_of(1.0f / sm.R[k], ketau, sc);
        } else {
            const float dx = sm.x[l] - sm.x[k], dy = sm.y[l] - sm.y[k], dz = sm.z[l] - sm.z[k];
            const float r2 = dx * dx + dy * dy + dz * dz;
            const float rinv = frsq(r2);
            const float ex = fexp_neg(0.25f * r2 / (sm.R[k] * sm.R[l]));
            const float finv = frsq(__builtin_fmaf(sm.R[k] * sm.R[l], ex, r2));
            K = (r2 < sc.cut2) ? ke_in * rinv - kg_of(finv, ketau, sc) : 0.0f;
        }
        quad += sm.d[k] * sm.d[l] * K;
    }
    return block_sum_d((double)lin + 0.5 * (double)quad, sm.red);
}

__device__ void load_site(SiteSmem& sm, int m, int slot0, int nw, int ms, int ntot,
                          const int32_t* __restrict__ site_atoms, const float* __restrict__ state_q,
                          const float* __restrict__ xyz, const float* __restrict__ q,
                          const float* __restrict__ R)
{
    for (int k = threadIdx.x; k < m; k += blockDim.x) {
        const int a = site_atoms[slot0 + k];
        sm.atom[k] = a;
        sm.x[k] = xyz[a]; sm.y[k] = xyz[ntot + a]; sm.z[k] = xyz[2 * ntot + a];
        sm.R[k] = R[a];
        sm.qn[k] = state_q[(int64_t)(slot0 + k) * ms + nw];
        sm.d[k] = sm.qn[k] - q[a];
    }
    __syncthreads();
}

// Candidate c = blockIdx.x is valid (a site in range, a state of that site,
// at most MAX_SITE atoms); m and the replica are returned.
__device__ bool candidate_ok(const gbr_sites& S, const int32_t* __restrict__ cand, int c, int n_rep,
                             int& site, int& nw, int& m, int& rep) {
    site = cand[2 * c];
    nw = cand[2 * c + 1];
    if (site < 0 || site >= S.n_sites) return false;
    m = S.site_off[site + 1] - S.site_off[site];
    rep = S.site_rep[site];
    return nw >= 0 && nw < S.n_states[site] && m <= MAX_SITE && m >= 1 && rep >= 0 && rep < n_rep;
}

// Chunk blockIdx.y of candidate blockIdx.x, added into dE_fx[c] (fixed point).
__global__ __launch_bounds__(TB) void k_titration(
    const int32_t* __restrict__ atom_off, int n_rep, int ntot, const float* __restrict__ xyz,
    const float* __restrict__ q, const float* __restrict__ R, gbr_sites S,
    const int32_t* __restrict__ cand, int n_cand, float ke_in, float ketau, Screening sc,
    int64_t* __restrict__ dE_fx, uint32_t* __restrict__ err)
{
    __shared__ SiteSmem sm;
    const int c = blockIdx.x;
    if (c >= n_cand) return;
    int site, nw, m = 0, rep = 0;
    if (!candidate_ok(S, cand, c, n_rep, site, nw, m, rep)) return;     // reported by k_titration_out
    const int a0 = atom_off[rep], n = atom_off[rep + 1] - a0;
    const int j0 = (int)blockIdx.y * TI_CHUNK;
    if (j0 >= n && blockIdx.y > 0) return;
    load_site(sm, m, S.site_off[site], nw, S.max_states, ntot, S.site_atoms, S.state_q, xyz, q, R);
    const double v = site_delta_e(sm, m, a0 + j0, a0 + min(n, j0 + TI_CHUNK), blockIdx.y == 0, ntot,
                                  xyz, q, R, ke_in, ketau, sc);
    if (threadIdx.x == 0) atomic_add_fx(&dE_fx[c], to_fixed(v, FX_ENERGY, err));
}

// dE[c] from its fixed-point sum (in place), or NaN and the site error bit for
// an invalid candidate.
__global__ void k_titration_out(int n_rep, gbr_sites S, const int32_t* __restrict__ cand,
                                int n_cand, double* __restrict__ dE, uint32_t* __restrict__ err)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n_cand) return;
    int site, nw, m = 0, rep = 0;
    int64_t* fx = reinterpret_cast<int64_t*>(dE);
    if (!candidate_ok(S, cand, c, n_rep, site, nw, m, rep)) {
        raise_error(err, GBR_ERR_SITE);
        dE[c] = __builtin_nan("");
        return;
    }
    dE[c] = from_fixed(fx[c], INV_FX_ENERGY);
}

__global__ void k_zero_i64_n(int64_t* __restrict__ p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

// Titration attempts, one site type at a time (protonation, then redox, so
// that the redox attempt sees the charges the protonation attempt left):
// k_mc_partial forms dE_elec of the replica's attempt chunk by chunk into
// acc_fx[rep], k_mc_decide takes the Metropolis decision:
//   dG = l dE - [G_ref(s') - G_ref(s)] + kT ln10 (pH - pKa_ref)(N_H(s') - N_H(s))   (pH)
//   dG = l dE - [G_ref(s') - G_ref(s)] + F (E - E0_ref)(N_e(s') - N_e(s))            (redox)
// (l: the replica's Hamiltonian scale) accepted iff dG <= 0 or u < exp(-dG/kT).
// Both kernels draw the same Philox words: word 0 picks the site among the
// replica's sites of the type, word 1 the new state, words 2-3 the uniform.
struct McPick {
    int site, nw;
    U4 w;
};

// Called by all 64 lanes of one wavefront (the result is the same in every
// lane): the replica's sites are scanned 64 at a time.
__device__ McPick mc_pick(const gbr_sites& S, const int32_t* __restrict__ site_state, int rep,
                          int type, uint64_t seed, uint64_t nstep) {
    McPick p{-1, 0, U4{0, 0, 0, 0}};
    const int lane = threadIdx.x & 63;
    const int s0 = S.rep_site_off[rep], s1 = S.rep_site_off[rep + 1];
    int cnt = 0;
    for (int k0 = s0; k0 < s1; k0 += 64) {
        const int k = k0 + lane;
        cnt += __popcll(__ballot(k < s1 && S.site_type[k] == type));
    }
    if (cnt == 0) return p;
    p.w = draw(seed, 0u, (uint32_t)rep, nstep, type == 0 ? STREAM_MCPH : STREAM_MCRED);
    const int pick = (int)choose(p.w.x, (uint32_t)cnt);
    const unsigned long long below = (1ull << lane) - 1ull;
    for (int k0 = s0, seen = 0; k0 < s1; k0 += 64) {
        const int k = k0 + lane;
        const bool mine = k < s1 && S.site_type[k] == type;
        const unsigned long long b = __ballot(mine);
        const int c = __popcll(b);
        if (pick < seen + c) {                 // the (pick - seen)-th site of this window
            const unsigned long long hit = __ballot(mine && __popcll(b & below) == pick - seen);
            p.site = k0 + __ffsll((long long)hit) - 1;
            break;
        }
        seen += c;
    }
    const int cur = site_state[p.site];
    const uint32_t off = choose(p.w.y, (uint32_t)(S.n_states[p.site] - 1));
    p.nw = (int)off < cur ? (int)off : (int)off + 1;
    return p;
}

// Chunk blockIdx.y of replica blockIdx.x.
__global__ __launch_bounds__(TB) void k_mc_partial(
    const int32_t* __restrict__ atom_off, int n_rep, int ntot, const uint64_t* __restrict__ step,
    uint64_t seed, int type, const float* __restrict__ xyz, const float* __restrict__ q,
    const float* __restrict__ R, gbr_sites S, const int32_t* __restrict__ site_state, float ke_in,
    float ketau, Screening sc, int64_t* __restrict__ acc_fx, uint32_t* __restrict__ err)
{
    __shared__ SiteSmem sm;
    __shared__ int s_site, s_new;
    const int rep = blockIdx.x;
    if (rep >= n_rep) return;
    const int a0 = atom_off[rep], n = atom_off[rep + 1] - a0;
    const int j0 = (int)blockIdx.y * TI_CHUNK;
    if (j0 >= n && blockIdx.y > 0) return;
    if (threadIdx.x < 64) {                 // wavefront 0 picks
        const McPick p = mc_pick(S, site_state, rep, type, seed, step[0]);
        if (threadIdx.x == 0) {
            const bool ok = p.site >= 0 && S.site_off[p.site + 1] - S.site_off[p.site] <= MAX_SITE;
            s_site = ok ? p.site : -1;
            s_new = p.nw;
        }
    }
    __syncthreads();
    const int site = s_site;
    if (site < 0) return;                 // no site of the type, or reported by k_mc_decide
    const int m = S.site_off[site + 1] - S.site_off[site];
    load_site(sm, m, S.site_off[site], s_new, S.max_states, ntot, S.site_atoms, S.state_q, xyz, q, R);
    const double v = site_delta_e(sm, m, a0 + j0, a0 + min(n, j0 + TI_CHUNK), blockIdx.y == 0, ntot,
                                  xyz, q, R, ke_in, ketau, sc);
    if (threadIdx.x == 0) atomic_add_fx(&acc_fx[rep], to_fixed(v, FX_ENERGY, err));
}

// One wavefront per replica: the decision, the new charges, the counters;
// clears acc_fx[rep] for the next attempt.
__global__ __launch_bounds__(64) void k_mc_decide(
    int n_rep, const uint64_t* __restrict__ step, uint64_t seed, int type, float* __restrict__ q,
    gbr_sites S, gbr_grid G, int32_t* __restrict__ site_state,
    const int32_t* __restrict__ target_idx, uint32_t* __restrict__ mc_stats,
    int64_t* __restrict__ acc_fx, uint32_t* __restrict__ err)
{
    const int rep = blockIdx.x;
    if (rep >= n_rep) return;
    const McPick p = mc_pick(S, site_state, rep, type, seed, step[0]);
    if (p.site < 0) return;
    const int site = p.site, nw = p.nw, ms = S.max_states;
    const int m = S.site_off[site + 1] - S.site_off[site];
    if (m > MAX_SITE) {
        if (threadIdx.x == 0) raise_error(err, GBR_ERR_SITE);
        return;
    }
    const int cur = site_state[site];
    const double dEel = from_fixed(acc_fx[rep], INV_FX_ENERGY);
    const int32_t* tg = target_idx + GBR_N_DIMS * rep;
    const double kT = KB * G.T_vals[tg[GBR_DIM_T]];
    const double lam = ham_scale(G.H_scale, target_idx, rep);
    double dG = lam * dEel - (S.G_ref[site * ms + nw] - S.G_ref[site * ms + cur]);
    if (type == 0) {
        const double pH = G.pH_vals[tg[GBR_DIM_PH]];
        dG += kT * LN10 * (pH - S.ref_value[site])
              * (double)(S.state_nH[site * ms + nw] - S.state_nH[site * ms + cur]);
    } else {
        const double Ev = G.E_vals[tg[GBR_DIM_E]];
        dG += FARADAY * (Ev - S.ref_value[site])
              * (double)(S.state_ne[site * ms + nw] - S.state_ne[site * ms + cur]);
    }
    const double u = uniform53(p.w.z, p.w.w);
    const bool acc = dG <= 0.0 || u < exp(-dG / kT);
    __syncthreads();                      // every lane has read site_state and acc_fx
    if (acc) {
        const int slot0 = S.site_off[site];
        for (int k = threadIdx.x; k < m; k += blockDim.x)
            q[S.site_atoms[slot0 + k]] = S.state_q[(int64_t)(slot0 + k) * ms + nw];
    }
    if (threadIdx.x == 0) {
        if (!(dG == dG)) raise_error(err, GBR_ERR_NONFINITE);
        if (acc) site_state[site] = nw;
        acc_fx[rep] = 0;
        if (mc_stats) {
            mc_stats[2 * site] += 1;
            if (acc) mc_stats[2 * site + 1] += 1;
        }
    }
}

// --------------------------------------------------------- replica exchange
// Per replica: protons, electrons, the energy entering the temperature
// exchange, U_l - sum G_ref(s) + sum_redox F (E - E0_ref) N_e(s)  (mode 0) or U_l
// (mode 1) with U_l = l (E_GB + E_C + E_LJ) + E_tether, and (enb, may be NULL)
// the unscaled E_GB + E_C + E_LJ that the Hamiltonian exchange compares.
__global__ void k_exchange_inputs(int n_rep, gbr_sites S, gbr_grid G,
                                  const int32_t* __restrict__ site_state,
                                  const int32_t* __restrict__ target_idx,
                                  const int64_t* __restrict__ energy_fx, int eps_mode,
                                  int32_t* __restrict__ nH, int32_t* __restrict__ ne,
                                  double* __restrict__ epsT, double* __restrict__ enb)
{
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n_rep) return;
    const int ms = S.max_states;
    int h = 0, e = 0;
    double extra = 0.0;
    const double Ev = G.E_vals[target_idx[GBR_N_DIMS * r + GBR_DIM_E]];
    if (S.rep_site_off) {
        for (int k = S.rep_site_off[r]; k < S.rep_site_off[r + 1]; ++k) {
            const int st = site_state[k];
            h += S.state_nH[k * ms + st];
            e += S.state_ne[k * ms + st];
            extra -= S.G_ref[k * ms + st];
            if (S.site_type[k] == GBR_SITE_REDOX)
                extra += FARADAY * (Ev - S.ref_value[k]) * (double)S.state_ne[k * ms + st];
        }
    }
    double W = 0.0;
    for (int c = 0; c < 3; ++c) W += from_fixed(energy_fx[4 * r + c], INV_FX_ENERGY);
    const double U = ham_scale(G.H_scale, target_idx, r) * W + from_fixed(energy_fx[4 * r + 3], INV_FX_ENERGY);
    nH[r] = h;
    ne[r] = e;
    epsT[r] = eps_mode == 0 ? U + extra : U;
    if (enb) enb[r] = W;
}

// One thread per grid point.  The attempt index is `attempt` or, when
// step_dev is given, (step + 1) / ex_every - 1 for the step being executed.
// fscale (may be NULL) receives l_new / l_old for replicas whose Hamiltonian
// level changed and 1 otherwise.
__global__ void k_exchange(gbr_grid G, uint64_t attempt, const uint64_t* __restrict__ step_dev,
                           int ex_every, const int32_t* __restrict__ nH,
                           const int32_t* __restrict__ ne, const double* __restrict__ epsT,
                           const double* __restrict__ enb, int32_t* __restrict__ target_idx,
                           int32_t* __restrict__ grid_rep, float* __restrict__ vscale,
                           double* __restrict__ fscale, uint32_t* __restrict__ ex_stats,
                           uint64_t seed)
{
    const int Gp = G.nE * G.npH * G.nT * G.nHam;
    const int gg = blockIdx.x * blockDim.x + threadIdx.x;
    if (gg >= Gp * G.n_inst) return;
    // step_dev[0] = n + 1 once the step's force evaluation and kick are done
    const uint64_t a = step_dev ? step_dev[0] / (uint64_t)ex_every - 1 : attempt;
    const int d = G.dim_order[a % (uint64_t)G.n_dims];
    const int parity = (int)((a / (uint64_t)G.n_dims) & 1);
    const int inst = gg / Gp, g = gg % Gp;
    const int c[GBR_N_DIMS] = {g / (G.npH * G.nT * G.nHam), (g / (G.nT * G.nHam)) % G.npH,
                               (g / G.nHam) % G.nT, g % G.nHam};
    const int sz[GBR_N_DIMS] = {G.nE, G.npH, G.nT, G.nHam};
    const int k = c[d];
    const bool lower = (k & 1) == parity && k + 1 < sz[d];
    const bool upper = k >= 1 && ((k - 1) & 1) == parity;
    const int ri = grid_rep[gg];
    if (!lower) {
        if (!upper) {
            vscale[ri] = 1.0f;
            if (fscale) fscale[ri] = 1.0;
        }
        return;
    }
    int c2[GBR_N_DIMS] = {c[0], c[1], c[2], c[3]};
    c2[d] = k + 1;
    const int gu = inst * Gp + ((c2[0] * G.npH + c2[1]) * G.nT + c2[2]) * G.nHam + c2[3];
    const int rj = grid_rep[gu];
    double delta;
    if (d == GBR_DIM_PH) {
        delta = LN10 * (G.pH_vals[k] - G.pH_vals[k + 1]) * (double)(nH[ri] - nH[rj]);
    } else if (d == GBR_DIM_E) {
        const double kT = KB * G.T_vals[c[GBR_DIM_T]];
        delta = FARADAY / kT * (G.E_vals[k] - G.E_vals[k + 1]) * (double)(ne[ri] - ne[rj]);
    } else if (d == GBR_DIM_T) {
        const double bi = 1.0 / (KB * G.T_vals[k]), bj = 1.0 / (KB * G.T_vals[k + 1]);
        delta = (bi - bj) * (epsT[ri] - epsT[rj]);
    } else {
        const double kT = KB * G.T_vals[c[GBR_DIM_T]];
        delta = (G.H_scale[k] - G.H_scale[k + 1]) / kT * (enb[ri] - enb[rj]);
    }
    const U4 w = draw(seed, 0u, (uint32_t)gg, a, STREAM_EX);
    const double u = uniform53(w.x, w.y);
    const bool acc = delta >= 0.0 || u < exp(delta);
    const int GT = Gp * G.n_inst;
    if (ex_stats) {
        ex_stats[d * GT + gg] += 1;
        if (acc) ex_stats[GBR_N_DIMS * GT + d * GT + gg] += 1;
    }
    float si = 1.0f, sj = 1.0f;
    double fi = 1.0, fj = 1.0;
    if (acc) {
        target_idx[GBR_N_DIMS * ri + d] = k + 1;
        target_idx[GBR_N_DIMS * rj + d] = k;
        grid_rep[gg] = rj;
        grid_rep[gu] = ri;
        if (d == GBR_DIM_T) {
            si = (float)sqrt(G.T_vals[k + 1] / G.T_vals[k]);
            sj = (float)sqrt(G.T_vals[k] / G.T_vals[k + 1]);
        } else if (d == GBR_DIM_H) {
            fi = G.H_scale[k + 1] / G.H_scale[k];
            fj = G.H_scale[k] / G.H_scale[k + 1];
        }
    }
    vscale[ri] = si;
    vscale[rj] = sj;
    if (fscale) {
        fscale[ri] = fi;
        fscale[rj] = fj;
    }
}

// After an exchange attempt: velocities of replicas whose temperature changed
// times vscale; with fscale, the forces of replicas whose Hamiltonian level
// changed made those of the new level: the pair part (the force less the
// tether term k_md_last added, the same integer) times l_new / l_old.
__global__ void k_apply_swaps(int ntot, int n_rep, const int32_t* __restrict__ atom_off,
                              const float* __restrict__ vscale, float* __restrict__ v,
                              const double* __restrict__ fscale, const float* __restrict__ xyz,
                              const float* __restrict__ x0, double k_t,
                              int64_t* __restrict__ force_fx, uint32_t* __restrict__ err)
{
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= ntot) return;
    int lo = 0, hi = n_rep;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (atom_off[mid] <= a) lo = mid; else hi = mid;
    }
    const float s = vscale[lo];
    if (s != 1.0f) {
        v[a] *= s;
        v[ntot + a] *= s;
        v[2 * ntot + a] *= s;
    }
    const double fs = fscale ? fscale[lo] : 1.0;
    if (fs != 1.0) {
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const int64_t idx = (int64_t)d * ntot + a;
            const double dx = (double)xyz[idx] - (double)x0[idx];
            const int64_t ft = to_fixed(-2.0 * k_t * dx, FX_FORCE, err);
            force_fx[idx] = scale_fx(force_fx[idx] - ft, fs, err) + ft;
        }
    }
}

int tile_grid(const gbr_ctx* c) { return (c->n_tiles + 3) / 4; }

}  // namespace

namespace gbr {

hipError_t launch_set_step(const gbr_ctx* c, uint64_t step0, hipStream_t s) {
    hipLaunchKernelGGL(k_set_step, dim3(1), dim3(1), 0, s, c->step, step0);
    return hipGetLastError();
}

hipError_t launch_md_first(const gbr_ctx* c, const MDArgs& a, bool mid, hipStream_t s) {
    const double hdt = 0.5 * a.pr.dt;
    const double c1 = exp(-a.pr.gamma * a.pr.dt);
    const double c2 = sqrt(1.0 - c1 * c1);
#define GBR_MDF(MID) hipLaunchKernelGGL(k_md_first<MID>, dim3(tile_grid(c)), dim3(256), 0, s, c->tiles, \
        c->n_tiles, c->atom_off, c->n_atoms, c->step, a.seed, hdt, c1, c2, a.pr.mass, a.pr.grid.T_vals, \
        a.pr.grid.H_scale, a.st.target_idx, a.st.xyz, a.st.v, a.st.force_fx, a.st.energy_fx, c->psi_fx, c->dEdR_fx, \
        c->ke_fx, a.st.ke, a.pr.x0, a.pr.k_tether, c->err)
    if (mid) GBR_MDF(true); else GBR_MDF(false);
#undef GBR_MDF
    return hipGetLastError();
}

hipError_t launch_md_last(const gbr_ctx* c, const MDArgs& a, int kick, hipStream_t s) {
    hipLaunchKernelGGL(k_md_last, dim3((c->n_tiles + 7) / 8), dim3(512), 0, s, c->tiles, c->n_tiles,
                       c->atom_off, c->n_atoms, 0.5 * a.pr.dt, a.pr.k_tether, a.pr.grid.H_scale,
                       a.st.target_idx, a.pr.mass, a.pr.x0, a.st.xyz, a.st.v, a.st.force_fx, a.st.energy_fx, c->ke_fx,
                       kick, c->err);
    return hipGetLastError();
}

hipError_t launch_ke_out(const gbr_ctx* c, double* ke, hipStream_t s) {
    if (!ke) return hipSuccess;
    hipLaunchKernelGGL(k_ke_out, dim3((c->n_rep + 255) / 256), dim3(256), 0, s, c->n_rep,
                       c->ke_fx, ke);
    return hipGetLastError();
}

Screening make_screening(const gbr_gb_params& p) {
    Screening sc;
    sc.keout = (float)(p.k_e / p.eps_out);
    sc.kappa = (float)p.kappa;
    sc.cut2 = p.cut > 0 ? (float)(p.cut * p.cut) : FLT_MAX;
    return sc;
}

static int ti_chunks(const gbr_ctx* c) { return (c->max_n + TI_CHUNK - 1) / TI_CHUNK; }

hipError_t launch_mc(const gbr_ctx* c, const MDArgs& a, hipStream_t s) {
    const GBConstH k = make_const(c->prm);
    const dim3 grid(c->n_rep, ti_chunks(c));
    for (int type = 0; type < 2; ++type) {
        hipLaunchKernelGGL(k_mc_partial, grid, dim3(TB), 0, s, c->atom_off, c->n_rep, c->n_atoms,
                           c->step, a.seed, type, a.st.xyz, a.st.q, a.st.R, a.pr.sites,
                           a.st.site_state, k.ke_in, (float)(k.ke_d * k.tau_d),
                           make_screening(c->prm), c->mc_acc_fx, c->err);
        hipLaunchKernelGGL(k_mc_decide, dim3(c->n_rep), dim3(64), 0, s, c->n_rep, c->step, a.seed,
                           type, a.st.q, a.pr.sites, a.pr.grid, a.st.site_state, a.st.target_idx,
                           a.st.mc_stats, c->mc_acc_fx, c->err);
    }
    return hipGetLastError();
}

hipError_t launch_titration(const gbr_ctx* c, const float* xyz, const float* q, const float* R,
                            const gbr_sites& sites, const int32_t* cand, int32_t n_cand,
                            double* dE, hipStream_t s) {
    if (n_cand <= 0) return hipSuccess;
    const GBConstH k = make_const(c->prm);
    int64_t* fx = reinterpret_cast<int64_t*>(dE);
    hipLaunchKernelGGL(k_zero_i64_n, dim3((n_cand + 255) / 256), dim3(256), 0, s, fx, n_cand);
    hipLaunchKernelGGL(k_titration, dim3(n_cand, ti_chunks(c)), dim3(TB), 0, s, c->atom_off, c->n_rep,
                       c->n_atoms, xyz, q, R, sites, cand, n_cand, k.ke_in,
                       (float)(k.ke_d * k.tau_d), make_screening(c->prm), fx, c->err);
    hipLaunchKernelGGL(k_titration_out, dim3((n_cand + 255) / 256), dim3(256), 0, s, c->n_rep, sites,
                       cand, n_cand, dE, c->err);
    return hipGetLastError();
}

hipError_t launch_exchange_inputs(const gbr_ctx* c, const gbr_md_state& st,
                                  const gbr_md_params& pr, int32_t* nH, int32_t* ne,
                                  double* epsT, double* enb, hipStream_t s) {
    hipLaunchKernelGGL(k_exchange_inputs, dim3((c->n_rep + 127) / 128), dim3(128), 0, s, c->n_rep,
                       pr.sites, pr.grid, st.site_state, st.target_idx, st.energy_fx, pr.eps_mode,
                       nH, ne, epsT, enb);
    return hipGetLastError();
}

hipError_t launch_exchange(const gbr_ctx* c, const gbr_grid& g, uint64_t attempt,
                           const uint64_t* attempt_from_step, int32_t ex_every,
                           const int32_t* nH, const int32_t* ne, const double* epsT,
                           const double* enb, int32_t* target_idx, int32_t* grid_rep,
                           float* vscale, double* fscale, uint32_t* ex_stats, uint64_t seed,
                           hipStream_t s) {
    (void)c;
    const int total = g.n_inst * g.nE * g.npH * g.nT * g.nHam;
    hipLaunchKernelGGL(k_exchange, dim3((total + 127) / 128), dim3(128), 0, s, g, attempt,
                       attempt_from_step, ex_every, nH, ne, epsT, enb, target_idx, grid_rep, vscale,
                       fscale, ex_stats, seed);
    return hipGetLastError();
}

hipError_t launch_apply_swaps(const gbr_ctx* c, const MDArgs& a, const float* vscale,
                              const double* fscale, hipStream_t s) {
    hipLaunchKernelGGL(k_apply_swaps, dim3((c->n_atoms + 255) / 256), dim3(256), 0, s,
                       c->n_atoms, c->n_rep, c->atom_off, vscale, a.st.v, fscale, a.st.xyz,
                       a.pr.x0, a.pr.k_tether, a.st.force_fx, c->err);
    return hipGetLastError();
}

}  // namespace gbr
