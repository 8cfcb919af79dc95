// gbr_internal.h -- host-side declarations shared by the library's
// translation units: the context layout and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "gbremd.h"

namespace gbr {

// Pair work list of one register blocking (items as in pair_list.h).
struct PairList {
    int ni = 0;                // i atoms per lane the list was built for
    int2* items = nullptr;     // {rep | type << 30, (A << 16) | B}
    int32_t n_items = 0;
    // with both cutoffs: the lists the passes run, for the descreening passes
    // (radius rgbmax, [0]) and for the energy pass (cut, [1]): the n_intra
    // items whose pairs lie inside one I block (a fixed prefix), then the
    // packed items of the current positions
    int2* run[2] = {nullptr, nullptr};
    int32_t* n_run[2] = {nullptr, nullptr};      // their counts (device)
    int32_t n_intra = 0;
    int2* iblk = nullptr;                        // I blocks {rep, A} with tiles after them
    int32_t* blk_p0 = nullptr;                   // [n_iblk] each block's first packed tile
    int32_t n_iblk = 0;
    int4* win = nullptr;                         // packing windows (pair_list.h PackWindow)
    int32_t n_win = 0;
    int32_t* blk_win = nullptr;                  // [n_iblk + 1] each block's first window
    int64_t pk_cap = 0;                          // packed tiles at most (tiles after each block)
    int32_t* blk_count[2] = {nullptr, nullptr};  // [n_iblk] atoms packed, zero between evaluations
    int32_t* pk_hdr[2] = {nullptr, nullptr};     // [pk_cap] A << 7 | nj
    int32_t* pk_j[2] = {nullptr, nullptr};       // [64 pk_cap] replica-local J atoms
};

struct LaunchShape {
    int waves_per_group = 4;
    int groups_per_cu = 8;
};

struct Timer {
    int32_t mask = 0;               // bit k: time kernels of kind k
    std::vector<hipEvent_t> pool;   // pairs of events
    std::vector<int> kind;          // kind of each recorded pair
    size_t used = 0;
    double ms[GBR_K_COUNT] = {0};
    int64_t count[GBR_K_COUNT] = {0};
};

}  // namespace gbr

// The energy pass adds each wavefront's energy sums into one of E_STRIPES
// cache lines of the replica rather than into its energy_fx slots: with one
// large replica, thousands of wavefronts end at about the same time, and adds
// to one address are served one after another.
constexpr int E_STRIPES = 32;
constexpr int E_STRIPE_LEN = 16;     // int64 per stripe: one 128-byte line

struct gbr_ctx {
    int device = 0;
    int n_cu = 256;
    gbr_gb_params prm{};
    int32_t n_rep = 0, n_atoms = 0, max_n = 0;
    int64_t n_pairs = 0;
    std::vector<int32_t> h_atom_off;
    int32_t* atom_off = nullptr;     // [n_rep+1]
    int2* tiles = nullptr;           // per-atom tiles {rep, tile}
    int32_t n_tiles = 0;
    gbr::PairList lists[4];          // NI = 1, 2, 4, 8
    bool packed = false;             // both cutoffs set: the pair passes run packed lists
    int32_t* tile_base = nullptr;    // [n_rep] index of each replica's first tile
    float4* tile_box = nullptr;      // [2 n_tiles] per-tile bounding boxes (min, max)
    int32_t* pack_count = nullptr;   // [8] items per list and radius
    int ni_born = 4, ni_energy = 4, ni_chain = 4;
    int split_den = 16;              // the last ceil(nb / split_den) block items of a replica run as halves
    gbr::LaunchShape shape;
    // workspace
    int64_t* psi_fx = nullptr;       // [N] sum_j h_ij (2^40)
    int64_t* dEdR_fx = nullptr;      // [N] pair part of dE/dR_i (2^40)
    double* dEdR = nullptr;          // [N] total dE/dR_i
    float* chain_c = nullptr;        // [N] (dE/dR)(dR/dpsi)(rho~/2)
    int64_t* ke_fx = nullptr;        // [n_rep] (2^32)
    int32_t* ex_nH = nullptr;        // [n_rep]
    int32_t* ex_ne = nullptr;
    double* ex_eps = nullptr;
    double* ex_enb = nullptr;        // [n_rep] unscaled GB + C + LJ energy
    float* ex_vscale = nullptr;
    double* ex_fscale = nullptr;     // [n_rep] force factor after Hamiltonian swaps
    int64_t* mc_acc_fx = nullptr;    // [n_rep] titration attempt dE (2^32), zero between attempts
    // [n_rep][E_STRIPES][E_STRIPE_LEN] energy-pass sums (E_GB, E_C, E_LJ at 2^32),
    // zero between evaluations: the energy pass adds into them, k_coef (always
    // the next launch) folds them into energy_fx and clears them
    int64_t* e_stripe = nullptr;
    uint64_t* step = nullptr;        // [2] current step index (second word unused)
    uint32_t* err = nullptr;         // device error word
    gbr::Timer timer;
    // captured per-step graphs (plain, MC, EX, MC+EX)
    hipGraphExec_t graph[16] = {};   // md_step graphs by step kind (mc, ex, mid head, last tail)
    uint64_t graph_key[16] = {};
    hipStream_t cap_stream = nullptr;
};

namespace gbr {

struct GBConstH {
    float ke, ke_in, tau, offset;
    double ke_d, ke_in_d, tau_d, offset_d, alpha, beta, gamma;
};
GBConstH make_const(const gbr_gb_params& p);

// kernel launchers (pair kernels) ----------------------------------------
// ev: timing events (start, stop) recorded by the kernel's own dispatch
// (hipExtLaunchKernel), or null.
struct LaunchEvents {
    hipEvent_t start = nullptr, stop = nullptr;
};
hipError_t launch_born_pair(const gbr_ctx* c, const float* xyz, const float* rho,
                            const float* screen, hipStream_t s, LaunchEvents ev = {});
hipError_t launch_energy_pair(const gbr_ctx* c, const float* xyz, const float* q,
                              const float* R, const float* sigma, const float* eps,
                              int64_t* force_fx, int64_t* dEdq_fx,
                              hipStream_t s, LaunchEvents ev = {});
hipError_t launch_chain_pair(const gbr_ctx* c, const float* xyz, const float* rho,
                             const float* screen, int64_t* force_fx, int64_t* dEdrho_fx,
                             hipStream_t s, LaunchEvents ev = {});

// The descreening pass without a context or list (gb_born_radii_noalloc):
// items generated from the wavefront index over max_tiles tiles per replica,
// NI = 1, the rgbmax cutoff when set; sums into psi_fx (zeroed by the caller).
hipError_t launch_born_pair_gen(const gbr_gb_params& p, int n_rep, int max_tiles, const int32_t* atom_off,
                                int n_atoms, int n_cu, const float* xyz, const float* rho,
                                const float* screen, int64_t* psi_fx, uint32_t* err, hipStream_t s);

// With both cutoffs: per-tile bounding boxes of xyz, then for every list in
// use and every I block the atoms after the block that come within rgbmax
// (for the descreening passes) or cut (for the energy pass) of its box,
// packed into items after the list's intra-block items.
hipError_t launch_pack(const gbr_ctx* c, const float* xyz, hipStream_t s);

// per-atom kernels ------------------------------------------------------------
hipError_t launch_zero_i64(int64_t* p, int64_t n, hipStream_t s);
hipError_t launch_born_finalize(const gbr_ctx* c, const float* rho, float* R, float* dRdpsi,
                                double* psi, hipStream_t s);
hipError_t launch_born_finalize_flat(const gbr_gb_params& p, int n_atoms, int n_rep,
                                     const int32_t* atom_off, const float* rho, const int64_t* psi_fx,
                                     float* R, float* dRdpsi, double* psi, uint32_t* err, hipStream_t s);
hipError_t launch_coef(const gbr_ctx* c, const float* q, const float* rho, const float* R,
                       const float* dRdpsi, int64_t* energy_fx, int64_t* dEdq_fx, uint64_t* step,
                       hipStream_t s);
hipError_t launch_rho_finalize(const gbr_ctx* c, const float* rho, const float* R,
                               const float* dRdpsi, const double* psi, int64_t* dEdrho_fx,
                               hipStream_t s);
hipError_t launch_energies(const gbr_ctx* c, const int64_t* e, double* out, hipStream_t s);
hipError_t launch_fx_to_float(const gbr_ctx* c, const int64_t* src, int comps, int bits,
                              const double* scale, int sign, float* dst, hipStream_t s);

// dynamics ---------------------------------------------------------------------
struct MDArgs {
    gbr_md_state st;
    gbr_md_params pr;
    uint64_t seed;
};
hipError_t launch_set_step(const gbr_ctx* c, uint64_t step0, hipStream_t s);
hipError_t launch_md_first(const gbr_ctx* c, const MDArgs& a, bool mid, hipStream_t s);
hipError_t launch_md_last(const gbr_ctx* c, const MDArgs& a, int kick, hipStream_t s);
hipError_t launch_ke_out(const gbr_ctx* c, double* ke, hipStream_t s);
hipError_t launch_mc(const gbr_ctx* c, const MDArgs& a, hipStream_t s);
hipError_t launch_titration(const gbr_ctx* c, const float* xyz, const float* q, const float* R,
                            const gbr_sites& sites, const int32_t* cand, int32_t n_cand,
                            double* dE, hipStream_t s);
hipError_t launch_exchange_inputs(const gbr_ctx* c, const gbr_md_state& st,
                                  const gbr_md_params& pr, int32_t* nH, int32_t* ne,
                                  double* epsT, double* enb, hipStream_t s);
hipError_t launch_exchange(const gbr_ctx* c, const gbr_grid& g, uint64_t attempt,
                           const uint64_t* attempt_from_step, int32_t ex_every,
                           const int32_t* nH, const int32_t* ne, const double* epsT,
                           const double* enb, int32_t* target_idx, int32_t* grid_rep,
                           float* vscale, double* fscale, uint32_t* ex_stats, uint64_t seed,
                           hipStream_t s);
// Velocity scaling after temperature swaps and force rescaling after
// Hamiltonian swaps (fscale may be NULL).
hipError_t launch_apply_swaps(const gbr_ctx* c, const MDArgs& a, const float* vscale,
                              const double* fscale, hipStream_t s);

}  // namespace gbr
