/*
 * gbremd.h -- C ABI of the batched Generalized-Born C(pH,E)MD / REMD library
 * for AMD Instinct MI355X (gfx950).
 *
 * The library evaluates, for every replica of a multidimensional
 * E x pH x T replica-exchange simulation (Cruzeiro & Roitberg,
 * arXiv:1809.07726), the GB implicit-solvent nonbonded work in one batched
 * launch per pass:
 *   - effective Born radii: the pairwise HCT descreening sum with the OBC
 *     tanh rescaling (the igb=2 model named in Calculation details,
 *     "Implicit Solvent Calculations");
 *   - GB + Coulomb + Lennard-Jones energy and forces, including the chain rule
 *     through dE/dR_i, and optionally dE/dq and dE/drho;
 *   - the electrostatic energy change that decides each protonation / redox
 *     Monte Carlo attempt (Theory, "Constant pH and Redox Potential Molecular
 *     Dynamics", eqs. 1-2);
 *   - a BAOAB Langevin step with the Monte Carlo attempts and the exchange
 *     attempts of eqs. 3-5 (Theory, "Multidimensional Replica Exchange MD").
 *
 * Conventions
 *   - Every entry point returns 0 (GBR_OK) or a negative GBR_E_* code;
 *     gbr_last_error() returns a thread-local message for the last failure.
 *   - Arrays passed in are owned by the caller; unless stated otherwise they
 *     are DEVICE pointers (hipMalloc / torch CUDA tensors) on the context's
 *     device, and every call taking a context must be made with that device
 *     current (otherwise GBR_E_INVAL, nothing launched).  The library never
 *     frees or reallocates caller memory.  It owns only the opaque gbr_ctx
 *     (workspace, work lists, graphs, timers).
 *   - All compute entry points are asynchronous on the caller's stream; only
 *     gbr_check, gbr_get_timing and gbr_ctx_destroy synchronize.
 *   - Host-checkable argument errors return GBR_E_INVAL before anything is
 *     launched.  Data-dependent faults (non-finite values, fixed-point
 *     overflow, non-positive Born radius, site index out of range) set bits in
 *     a device error word that gbr_check() reads and clears.
 *   - Batch layout: replicas are stored back to back.  Replica r owns flat
 *     atoms atom_off[r] .. atom_off[r+1]-1 (atom_off given on the host at
 *     context creation).  Per-atom float arrays have n_atoms entries;
 *     coordinate-like arrays are SoA of 3 * n_atoms: x[0..N), y[N..2N), z[2N..3N).
 *   - Units: A, e, kcal/mol, amu, ps, K, V.
 *   - Accumulated outputs are 64-bit fixed point (value * 2^bits, round to
 *     nearest even), so results are bit-identical run to run for a given
 *     binary, register blocking and input, also with both cutoffs set (the
 *     packed cutoff lists place every atom by the coordinates alone).
 */
#ifndef GBREMD_H
#define GBREMD_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------- status codes */
#define GBR_OK           0
#define GBR_E_INVAL     (-1)  /* bad argument (null pointer, size, layout)      */
#define GBR_E_HIP       (-2)  /* a HIP runtime call failed                      */
#define GBR_E_NOMEM     (-3)  /* workspace allocation failed                    */
#define GBR_E_NODEVICE  (-4)  /* no usable gfx950 device                        */
#define GBR_E_NUMERIC   (-5)  /* gbr_check: the device error word was non-zero  */

/* device error-word bits (gbr_check) */
#define GBR_ERR_NONFINITE  0x1u  /* a pair or per-atom value was NaN or Inf      */
#define GBR_ERR_OVERFLOW   0x2u  /* a fixed-point conversion saturated           */
#define GBR_ERR_RADIUS     0x4u  /* 1/R_i <= 0 or not finite                     */
#define GBR_ERR_SITE       0x8u  /* titration candidate out of range             */
#define GBR_ERR_LAYOUT     0x10u /* gb_born_radii_noalloc: atom_off disagrees with
                                    n_atoms / max_atoms (replica skipped)       */

/* fixed-point scales: stored integer = round(value * 2^bits) */
#define GBR_FX_BITS_FORCE   40   /* forces, dE/dR, dE/dq, dE/drho (per atom)     */
#define GBR_FX_BITS_ENERGY  32   /* energies (per replica)                       */

/* gb_energy_forces flags */
#define GBR_GRAD_Q    0x1   /* also accumulate dE/dq into dEdq_fx                */
#define GBR_GRAD_RHO  0x2   /* also accumulate dE/drho into dEdrho_fx            */
#define GBR_ZERO_OUT  0x4   /* zero every output before accumulating into it    */

/* md_step flags */
#define GBR_MD_INIT_FORCES 0x1  /* compute forces/energies at xyz before step 1 */
#define GBR_MD_GRAPH       0x2  /* replay per-step HIP graphs (captured on first use) */

/* site types and exchange dimensions */
#define GBR_SITE_PH     0
#define GBR_SITE_REDOX  1
#define GBR_DIM_E   0
#define GBR_DIM_PH  1
#define GBR_DIM_T   2
#define GBR_DIM_H   3   /* Hamiltonian: scale of the GB + Coulomb + LJ energy */
#define GBR_N_DIMS  4

/* timed kernel kinds (gbr_get_timing) */
#define GBR_K_BORN_PAIR   0   /* descreening pair pass                        */
#define GBR_K_ENERGY_PAIR 1   /* energy / direct-force pair pass              */
#define GBR_K_CHAIN_PAIR  2   /* chain-rule pair pass                         */
#define GBR_K_PER_ATOM    3   /* every per-atom kernel                        */
#define GBR_K_TITRATION   4   /* titration energy change / Monte Carlo        */
#define GBR_K_EXCHANGE    5   /* exchange attempt                             */
#define GBR_K_COUNT       6

typedef struct gbr_ctx gbr_ctx;

#define GBR_MAX_ATOMS (1 << 28)   /* atoms of one batch (gbr_ctx_create) */

/* Generalized Born model constants.  OBC-II (igb=2): k_e = 332.0522173,
 * eps_in = 1, eps_out = 78.5, offset = 0.09 A, (alpha, beta, gamma) =
 * (1.0, 0.8, 4.85).  Optional (0 = off, the paper's setting):
 *   kappa  Debye-Hueckel screening of the GB term: a GB pair term is
 *          -k_e q_i q_j g(f_ij), a self term -(1/2) k_e q_i^2 g(R_i), with
 *          g(f) = (1/eps_in - exp(-kappa f)/eps_out) / f;
 *   cut    pairs at r >= cut drop out of the Coulomb, GB and LJ energies and
 *          of the titration energy changes (plain truncation);
 *   rgbmax pairs at r >= rgbmax drop out of the descreening sum.
 * Self terms always stay.  Forces are the gradients of the truncated sums. */
typedef struct {
    double k_e;       /* Coulomb constant, kcal A / (mol e^2)  */
    double eps_in;    /* solute dielectric                      */
    double eps_out;   /* solvent dielectric                     */
    double offset;    /* dielectric offset delta (A)            */
    double alpha, beta, gamma;
    double kappa;     /* 1/A, >= 0                              */
    double cut;       /* A, >= 0                                */
    double rgbmax;    /* A, >= 0                                */
} gbr_gb_params;

/* Titratable sites (Theory, C(pH,E)MD: a residue's protonation or redox state
 * is a set of atomic charges).  Sites are per replica and stored replica by
 * replica.  All pointers are device pointers.  max_states is the stride of the
 * per-state tables (2..8). */
typedef struct {
    int32_t n_sites;
    int32_t max_states;
    const int32_t* rep_site_off; /* [n_rep+1] sites of replica r: rep_site_off[r]..   */
    const int32_t* site_off;     /* [n_sites+1] site s owns slots site_off[s]..        */
    const int32_t* site_atoms;   /* [slots] flat atom index of each slot               */
    const int32_t* site_rep;     /* [n_sites] owning replica                            */
    const int32_t* site_type;    /* [n_sites] GBR_SITE_PH or GBR_SITE_REDOX             */
    const int32_t* n_states;     /* [n_sites] 2..max_states                             */
    const float*   state_q;      /* [slots * max_states] charge of slot k in state t    */
    const int32_t* state_nH;     /* [n_sites * max_states] protons in each state         */
    const int32_t* state_ne;     /* [n_sites * max_states] electrons in each state       */
    const double*  G_ref;        /* [n_sites * max_states] reference energy, kcal/mol   */
    const double*  ref_value;    /* [n_sites] pKa_ref (pH site) or E0_ref in V (redox)  */
} gbr_sites;

/* Replica grid: n_inst independent grids of nE x npH x nT x nHam target
 * points; grid point g = ((iE * npH + ipH) * nT + iT) * nHam + iH; replicas
 * sharing a grid instance exchange targets.  Value tables are device
 * pointers.  The Hamiltonian dimension (Theory: multidimensional REMD may
 * combine H-REMD with the others) is a family of potentials
 *   U_l(x) = l (E_GB + E_C + E_LJ)(x) + E_tether(x)
 * with one scale l = H_scale[iH] per level; nHam = 1 with H_scale NULL
 * means l = 1 for every replica. */
typedef struct {
    int32_t n_inst, nE, npH, nT, nHam;
    const double* E_vals;     /* [nE]  V  */
    const double* pH_vals;    /* [npH]    */
    const double* T_vals;     /* [nT]  K  */
    const double* H_scale;    /* [nHam] > 0, or NULL when nHam = 1 */
    int32_t n_dims;           /* 1..4: dimensions cycled by exchange attempts */
    int32_t dim_order[4];     /* GBR_DIM_* in attempt order                   */
} gbr_grid;

/* ------------------------------------------------------------------ context */

/* Create a context for one batch layout on the current HIP device.
 * atom_off_host: HOST array [n_rep+1], atom_off[0] = 0, non-decreasing, every
 * replica with at least 1 and at most 64 x 65535 atoms; 1 <= n_rep < 2^26;
 * at most GBR_MAX_ATOMS atoms in all (3 x n_atoms indexes fit int32).
 * Allocates the workspace (a few int64/float per atom, 4 KiB per replica
 * for the energy pass's partial sums, the pair work lists; with both cutoffs
 * set also the packed lists, up to 2 x 256 bytes per later tile of every I
 * block and blocking, which the pair passes rebuild from the positions at
 * every evaluation).  Errors:
 * GBR_E_INVAL, GBR_E_NODEVICE, GBR_E_NOMEM, GBR_E_HIP. */
int gbr_ctx_create(gbr_ctx** out, const gbr_gb_params* params, int32_t n_rep,
                   const int32_t* atom_off_host);

/* Synchronize the device and release everything the context owns; a null
 * ctx is a no-op that returns GBR_OK. */
int gbr_ctx_destroy(gbr_ctx* ctx);

/* Read (and clear) the device error word after synchronizing `stream`.
 * Returns GBR_OK, or GBR_E_NUMERIC with *bits_out set to the GBR_ERR_* bits
 * (bits_out may be NULL). */
int gbr_check(gbr_ctx* ctx, hipStream_t stream, uint32_t* bits_out);

/* Thread-local description of the last failure of any entry point. */
const char* gbr_last_error(void);

/* Total atoms and replicas of the context's batch. */
int gbr_ctx_sizes(const gbr_ctx* ctx, int32_t* n_atoms, int32_t* n_rep, int64_t* n_pairs);

/* Pair-kernel launch shape: waves per workgroup (1, 2 or 4) and workgroups per
 * compute unit for the persistent grid (1..32).  Defaults 4 and 8.  The shape
 * changes no result; captured md_step graphs are dropped and recaptured with
 * the new shape on next use. */
int gbr_set_launch(gbr_ctx* ctx, int32_t waves_per_group, int32_t groups_per_cu);

/* Register blocking of the three pair passes: i atoms held per lane (1, 2, 4
 * or 8) for the descreening, energy and chain-rule passes.  Defaults are
 * chosen from the largest replica at context creation. */
int gbr_set_blocking(gbr_ctx* ctx, int32_t ni_born, int32_t ni_energy, int32_t ni_chain);

/* Split level of the pair work lists: the last ceil(nb / split_den) of each
 * replica's nb block items run as two half items (rotation steps 0..31 and
 * 32..63), 1 <= split_den <= 1024 (default 16; 1 halves every block item, so
 * that a small batch has more, shorter items for the chip's wavefront slots).
 * Rebuilds the lists (synchronizes the device) and drops captured md_step
 * graphs.  Results are bit-reproducible for one split level, blocking and
 * input; another split level changes the FP32 rounding of per-item sums. */
int gbr_set_split(gbr_ctx* ctx, int32_t split_den);

/* Kernel timing with HIP events for every kernel of the GBR_K_* kinds whose
 * bit (1 << kind) is set in kinds_mask (0 disables; eager launches only:
 * md_step does not replay graphs while any kind is timed).  The pair kernels'
 * events come from their own dispatch (hipExtLaunchKernel) and time the kernel
 * alone; the other kinds' events are recorded on the launch stream around the
 * launch. */
int gbr_set_timing(gbr_ctx* ctx, int32_t kinds_mask);
/* Synchronizes; ms_out[k] = summed milliseconds, count_out[k] = launches, for
 * k < GBR_K_COUNT; then resets the accumulators. */
int gbr_get_timing(gbr_ctx* ctx, double* ms_out, int64_t* count_out);

/* --------------------------------------------------------------- the path */

/* Effective Born radii of the OBC generalized Born model (igb=2), the solvent
 * model of MD and of every titration attempt (Calculation details, "Implicit
 * Solvent Calculations"); the paper names the model, the formulas are the
 * published HCT descreening integral with the OBC rescaling:
 *   psi_i   = rho~_i * (1/2) sum_{j != i} h(r_ij; rho~_i, S_j rho~_j),  rho~ = rho - offset
 *   1/R_i   = 1/rho~_i - tanh(alpha psi_i - beta psi_i^2 + gamma psi_i^3) / rho_i
 *   dRdpsi_i = R_i^2 (1 - tanh^2) (alpha - 2 beta psi_i + 3 gamma psi_i^2) / rho_i
 * over all pairs of the same replica (no cutoff).  Pair terms in FP32, the
 * per-atom sum in 64-bit fixed point, the rescaling in FP64.
 * In:  xyz [3N] SoA, rho [N] intrinsic radii (> offset), screen [N] S_i.
 * Out: R [N], dRdpsi [N] (float); psi [N] (double, may be NULL).
 * Coincident atoms (r = 0) are not supported (non-finite -> error bit). */
int gb_born_radii(gbr_ctx* ctx, const float* xyz, const float* rho, const float* screen,
                  float* R, float* dRdpsi, double* psi, hipStream_t stream);

/* GB + Coulomb + Lennard-Jones energy and forces of every replica at given
 * Born radii (from gb_born_radii on the same xyz/rho/screen): the implicit-
 * solvent potential of the MD (Calculation details, "Implicit Solvent
 * Calculations", igb=2; all pairs, no exclusions, Lorentz-Berthelot LJ):
 *   E_GB = -k_e tau [ sum_{i<j} q_i q_j / f_ij + (1/2) sum_i q_i^2 / R_i ],
 *          tau = 1/eps_in - 1/eps_out, f_ij = sqrt(r^2 + R_i R_j exp(-r^2 / (4 R_i R_j)))
 *   E_C  = (k_e / eps_in) sum_{i<j} q_i q_j / r_ij
 *   E_LJ = sum_{i<j} 4 eps_ij [(sigma_ij / r)^12 - (sigma_ij / r)^6],
 *          sigma_ij = (sigma_i + sigma_j)/2, eps_ij = sqrt(eps_i eps_j)
 * Forces F = -dE/dx include the chain rule through the Born radii
 * (dE/dR_i -> dR_i/dpsi_i -> dpsi_i/dx).
 * In:  xyz [3N], q, rho, screen, sigma, eps, R, dRdpsi [N]; psi [N] (required
 *      only with GBR_GRAD_RHO).
 * Out (accumulated, fixed point): force_fx [3N] (2^40 per kcal/mol/A);
 *      energy_fx [4 n_rep] = {E_GB, E_C, E_LJ, untouched} (2^32 per kcal/mol);
 *      with GBR_GRAD_Q: dEdq_fx [N] (2^40 per kcal/mol/e);
 *      with GBR_GRAD_RHO: dEdrho_fx [N] (2^40 per kcal/mol/A), derivative with
 *      respect to the intrinsic radius at fixed S_i and sigma_i.
 * With GBR_ZERO_OUT the outputs are cleared first (on the stream, by kernel). */
int gb_energy_forces(gbr_ctx* ctx, const float* xyz, const float* q, const float* rho,
                     const float* screen, const float* sigma, const float* eps,
                     const float* R, const float* dRdpsi, const double* psi,
                     int64_t* force_fx, int64_t* energy_fx, int32_t flags,
                     int64_t* dEdq_fx, int64_t* dEdrho_fx, hipStream_t stream);

/* Electrostatic energy change of titration candidates at fixed Born radii:
 * the energy term of the Metropolis test of a protonation or redox attempt
 * (Theory, "Constant pH and Redox Potential Molecular Dynamics": a change of
 * protonation or redox state is a change of the site's charges, accepted
 * with the weights whose stationary fractions are eqs. 1 and 2):
 *   dE = sum_{k in S} d_k (K q)_k + (1/2) sum_{k,l in S} d_k d_l K_kl,
 *   K_ij = k_e (1/(eps_in r_ij) - tau / f_ij) (i != j), K_ii = -k_e tau / R_i,
 * where S is the candidate site's atoms and d = (charges of the new state) - q.
 * This equals E_elec(q') - E_elec(q) of the energy above without LJ.
 * cand: DEVICE int32 [2 n_cand] = (site, new_state) pairs.  Out: dE [n_cand]
 * (double, kcal/mol).  Pair terms FP32, totals FP64.  Sites are limited to
 * 64 atoms.  Out-of-range candidates set GBR_ERR_SITE and yield NaN. */
int titration_delta_e(gbr_ctx* ctx, const float* xyz, const float* q, const float* R,
                      const gbr_sites* sites, const int32_t* cand, int32_t n_cand,
                      double* dE, hipStream_t stream);

/* One replica-exchange attempt (eqs. 3-5, and the Hamiltonian exchange of
 * H-REMD).  Attempt index a selects the dimension dim_order[a % n_dims] and
 * the parity (a / n_dims) % 2; grid points k and k+1 along that dimension (k
 * of that parity) are paired within every line of equal other targets;
 * replica i holds point k, j point k+1.  Log acceptance:
 *   pH: ln10 (pH_k - pH_k+1)(N_H,i - N_H,j)
 *   E : F/(kB T) (E_k - E_k+1)(N_e,i - N_e,j)
 *   T : (1/(kB T_k) - 1/(kB T_k+1)) (epsT_i - epsT_j)
 *   H : (l_k - l_k+1)/(kB T) (enb_i - enb_j),  T, E, pH those of the line
 * accepted iff >= 0 or u < exp(.), u from Philox4x32-10(seed; ctr = {0, global
 * lower grid point, a, 4 << 24}).  Accepted pairs swap their target index and
 * grid_rep entries.  vscale [n_rep] receives sqrt(T_new / T_old) for replicas
 * whose temperature changed and 1 otherwise (the caller scales velocities).
 * In: nH, ne [n_rep] int32; epsT [n_rep] double; enb [n_rep] double, the
 * unscaled E_GB + E_C + E_LJ (read by H attempts only; may be NULL when the
 * grid has nHam = 1).  In/out: target_idx [4 n_rep] (iE, ipH, iT, iH), grid_rep
 * [n_inst * G].  ex_stats (may be NULL): [2 * 4 * n_inst * G] uint32 attempts
 * then accepts, indexed dim * n_inst G + global lower grid point. */
int remd_exchange(gbr_ctx* ctx, const gbr_grid* grid, uint64_t attempt,
                  const int32_t* nH, const int32_t* ne, const double* epsT, const double* enb,
                  int32_t* target_idx, int32_t* grid_rep, float* vscale,
                  uint32_t* ex_stats, uint64_t seed, hipStream_t stream);

/* MD state and parameters for md_step (device pointers inside). */
typedef struct {
    float*    xyz;         /* [3N] positions, in/out                               */
    float*    v;           /* [3N] velocities A/ps, in/out                         */
    float*    q;           /* [N] charges, in/out (titration updates site atoms)   */
    int64_t*  force_fx;    /* [3N] forces of U_l at xyz, in/out (2^40)             */
    int64_t*  energy_fx;   /* [4 n_rep] GB, C, LJ (unscaled), tether at xyz (2^32) */
    float*    R;           /* [N] Born radii at xyz, out                           */
    float*    dRdpsi;      /* [N] out                                               */
    int32_t*  site_state;  /* [n_sites] in/out                                      */
    int32_t*  target_idx;  /* [4 n_rep] in/out                                     */
    int32_t*  grid_rep;    /* [n_inst G] in/out                                    */
    double*   ke;          /* [n_rep] kinetic energy after the step, may be NULL   */
    uint32_t* mc_stats;    /* [2 n_sites] attempts then accepts, may be NULL       */
    uint32_t* ex_stats;    /* see remd_exchange, may be NULL                       */
} gbr_md_state;

typedef struct {
    const float* rho;
    const float* screen;
    const float* sigma;
    const float* eps;
    const float* mass;     /* [N] amu                                   */
    const float* x0;       /* [3N] tether sites                          */
    double k_tether;       /* E_tether = k |x - x0|^2                    */
    double dt;             /* ps                                          */
    double gamma;          /* Langevin friction 1/ps                      */
    int32_t mc_every;      /* titration attempts every mc_every steps (0: never) */
    int32_t ex_every;      /* exchange attempts every ex_every steps (0: never)  */
    int32_t eps_mode;      /* T-exchange energy: 0 semi-grand, 1 potential only  */
    gbr_sites sites;
    gbr_grid grid;
} gbr_md_params;

/* n_steps BAOAB Langevin steps of every replica at its current temperature
 * target (step indices step0 .. step0+n_steps-1): C(pH,E)MD with replica
 * exchange (Theory: MD halted for a protonation then a redox attempt;
 * exchanges along one dimension at a time, eqs. 3-5; Calculation details:
 * Langevin dynamics, here with the BAOAB splitting).  Step n: B (half kick with
 * the forces in state), A (half drift), O (exact Ornstein-Uhlenbeck at
 * T[iT], Philox normals), A; if (n+1) % mc_every == 0: Born radii at the new
 * positions, one protonation attempt then one redox attempt per replica
 * (uniformly chosen site of that type, uniformly chosen other state,
 * Metropolis on l dE - dG_ref + kT ln10 (pH - pKa_ref) dN_H or
 * + F (E - E0_ref) dN_e); forces of U_l = l (GB + C + LJ) + tether
 * k |x - x0|^2 at the new positions, l the replica's Hamiltonian scale; B;
 * then if (n+1) % ex_every == 0 exchange attempt (n+1)/ex_every - 1 with
 * epsT = U_l - sum G_ref + sum_redox F (E - E0_ref) N_e (eps_mode 0) or U_l
 * (eps_mode 1), and velocities scaled after T swaps.
 * Random numbers: Philox4x32-10 (Salmon et al., SC'11), key = {seed low 32,
 * seed high 32}, counter = {sub, entity, step low 32, stream << 24 | step bits
 * 32..55}: stream 1 = O-step noise (entity = replica, sub = 2 * local atom + 0/1,
 * Box-Muller on two 53-bit uniforms each), 2 = protonation attempt and 3 =
 * redox attempt (entity = replica, sub = 0: word 0 picks the site, word 1 the
 * new state, words 2-3 the acceptance uniform), 4 = exchange (entity = global
 * lower grid point, step = attempt index).
 * Consecutive steps with no exchange attempt between them share one kernel
 * (the closing tether and half kick of step n with the opening stages of step
 * n+1, same roundings); the state after the call, ke included, is that of the
 * last step.
 * Flags: GBR_MD_INIT_FORCES, GBR_MD_GRAPH. */
int md_step(gbr_ctx* ctx, gbr_md_state* state, const gbr_md_params* params,
            uint64_t seed, uint64_t step0, int32_t n_steps, int32_t flags,
            hipStream_t stream);

/* For callers that cannot allocate device memory (code under HIP stream
 * capture, tight serving loops, harnesses that forbid hipMalloc): the Born
 * radii of gb_born_radii without a context.  The descreening sums go to a
 * static device array of GBR_NOALLOC_MAX_ATOMS 64-bit integers (8 MiB), one
 * per device, held until the process ends; the call allocates nothing.
 *   params    GB constants as for gbr_ctx_create (HOST pointer); rgbmax is
 *             honoured, kappa and cut do not enter the Born radii
 *   atom_off  DEVICE int32 [n_rep+1], replica r owns atoms atom_off[r] ..
 *             atom_off[r+1]-1, atom_off[0] = 0, atom_off[n_rep] = n_atoms
 *   n_atoms   1 .. GBR_NOALLOC_MAX_ATOMS (larger: GBR_E_INVAL, nothing launched)
 *   max_atoms size of the largest replica (it sizes the launch); a replica
 *             larger than max_atoms, or atom_off ending elsewhere than
 *             n_atoms, sets GBR_ERR_LAYOUT in *err and that replica's radii
 *             are not valid
 *   xyz, rho, screen, R, dRdpsi, psi as for gb_born_radii (psi may be NULL)
 *   err       DEVICE uint32, GBR_ERR_* bits are OR-ed into it (the caller
 *             clears it and reads it after synchronizing the stream)
 * All pairs of a replica, one i tile against one j tile per wavefront: the
 * results equal gb_born_radii's within FP32 rounding of the per-tile sums.
 * Every call on a device uses that device's one array: calls that overlap
 * on one device (other streams, other threads) race and give wrong radii.
 * The first call on a device, or gbr_ctx_create on it, looks the array up
 * (no allocation); make that first call outside stream capture. */
#define GBR_NOALLOC_MAX_ATOMS (1 << 20)
int gb_born_radii_noalloc(const gbr_gb_params* params, int32_t n_rep, const int32_t* atom_off,
                          int32_t n_atoms, int32_t max_atoms, const float* xyz, const float* rho,
                          const float* screen, float* R, float* dRdpsi, double* psi,
                          uint32_t* err, hipStream_t stream);

/* ------------------------------------------------------------- utilities */

/* dst[i] = sign * scale[rep(i)] * src[i] / 2^bits for a fixed-point array of
 * `components` blocks of N per-atom values (components = 3 for SoA forces, 1
 * for per-atom scalars); scale may be NULL (1).  sign is +1 or -1. */
int gbr_fx_to_float(gbr_ctx* ctx, const int64_t* src, int32_t components, int32_t bits,
                    const double* scale, int32_t sign, float* dst, hipStream_t stream);

/* Energies as doubles: out[5 r + c] = energy_fx[4 r + c] / 2^32 for c < 4 and
 * out[5 r + 4] = E_GB + E_C + E_LJ of replica r. */
int gbr_energies(gbr_ctx* ctx, const int64_t* energy_fx, double* out, hipStream_t stream);

/* Per-replica exchange inputs from the current state: protons, electrons,
 * the T-exchange energy and the unscaled E_GB + E_C + E_LJ (as md_step
 * computes them; enb may be NULL). */
int gbr_exchange_inputs(gbr_ctx* ctx, const gbr_md_state* state, const gbr_md_params* params,
                        int32_t* nH, int32_t* ne, double* epsT, double* enb, hipStream_t stream);

#ifdef __cplusplus
}
#endif
#endif /* GBREMD_H */
