/*
 * gbr_oracle.c -- plain double-precision CPU oracle for the batched
 * Generalized-Born C(pH,E)MD / multidimensional-REMD hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library calls, links or
 * loads this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no code, header, table or constant with the HIP
 * path: every constant below is written out here from its published source.
 *
 * What is computed, and where it comes from:
 *   - Solvent model: the Onufriev-Bashford-Case generalized Born model that the
 *     paper uses in MD and in every protonation/redox attempt (Calculation
 *     details, "Implicit Solvent Calculations", igb=2).  The paper names the
 *     model only; its formulas are the published HCT pairwise descreening
 *     integral with the OBC tanh rescaling ("OBC-II": alpha, beta, gamma =
 *     1.0, 0.8, 4.85, dielectric offset 0.09 A) and Still's GB pair function.
 *   - Monte Carlo titration: discrete charge states, protonation attempt first
 *     then redox (Theory: C(pH,E)MD); the acceptance weights are those whose
 *     stationary fractions are eq. 1 (pH) and eq. 2 (redox potential).
 *   - Replica exchange: eq. 3 (pH), eq. 4 (E), eq. 5 (T); one dimension per
 *     attempt, cycled in a user order, nearest neighbours only, among replicas
 *     sharing the other targets (Theory: AMBER's multidimensional REMD module).
 *     A fourth, Hamiltonian dimension (H-REMD, which the same module may
 *     combine with the others) holds a family of potentials U_l = l (E_GB +
 *     E_C + E_LJ) + E_tether; its exchanges use the Metropolis rule for two
 *     replicas trading Hamiltonians at one temperature.
 *   - Dynamics: Langevin (Calculation details) integrated with the BAOAB
 *     splitting of Leimkuhler and Matthews.
 *   - Random numbers: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11).
 *
 * Everything is O(N^2) double loops in the order of the definitions; no
 * tiling, no fixed point, no fast math.  Parallel loops (OpenMP) are over
 * independent output rows only, each row summed serially in index order.
 *
 * Parity unpinned (definitional, checked by eye against the published model):
 * three choices of the GB model that no closed form, limit or invariant
 * separates from a close variant -- the signs of the OBC-II polynomial
 * (alpha psi - beta psi^2 + gamma psi^3), the 4 in Still's exp(-r^2 / (4 Ri
 * Rj)), and the Lorentz-Berthelot combination (arithmetic sigma, geometric
 * epsilon) of the Lennard-Jones pair.  Every other part is pinned by the
 * tests: closed forms, quadrature, limits (the R -> rho rho~ / offset
 * saturation among them), invariants, finite differences, enumerations and
 * sampled distributions (eq. 5's exchange energy under titration among them).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ---------------------------------------------------------------- constants */
#define ORC_KB    0.001987204259   /* Boltzmann constant, kcal/(mol K) (CODATA 2018 R / 4184) */
#define ORC_FARAD 23.0605480       /* Faraday constant, kcal/(mol V) (CODATA 2018 F / 4184)   */
#define ORC_LN10  2.302585092994045684
#define ORC_CONV  418.4            /* 1 kcal/(mol A amu) expressed in A/ps^2                   */
#define ORC_TWO_PI 6.283185307179586477

enum { ORC_STREAM_O = 1, ORC_STREAM_MCPH = 2, ORC_STREAM_MCRED = 3, ORC_STREAM_EX = 4 };
enum { ORC_DIM_E = 0, ORC_DIM_PH = 1, ORC_DIM_T = 2, ORC_DIM_H = 3, ORC_NDIM = 4 };

typedef struct {
    double k_e;      /* Coulomb constant, kcal A / (mol e^2)             */
    double eps_in;   /* solute dielectric                                 */
    double eps_out;  /* solvent dielectric                                */
    double offset;   /* dielectric offset delta: rho~ = rho - delta (A)   */
    double alpha, beta, gamma;  /* OBC rescaling coefficients             */
    double kappa;    /* Debye-Hueckel screening parameter (1/A), 0: no salt */
    double cut;      /* pair energy cutoff (A), 0: none                     */
    double rgbmax;   /* descreening cutoff (A), 0: none                     */
} orc_gb;

/* ===================================================== Philox4x32-10 (SC'11) */
/* One Philox round: two 32x32->64 multiplies by the published multipliers,
 * the high halves xored with the other counter words and the key. Ten rounds,
 * the key bumped by the published Weyl constants between rounds. */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Counter layout used by every random draw of the method:
 *   ctr = { sub-index, entity (replica or grid point), step low 32 bits,
 *           stream id << 24 | step bits 32..55 },  key = { seed low, seed high }. */
static void orc_draw(uint64_t seed, uint32_t sub, uint32_t entity, uint64_t step,
                     uint32_t stream, uint32_t out[4])
{
    uint32_t ctr[4] = { sub, entity, (uint32_t)step,
                        (stream << 24) | (uint32_t)((step >> 32) & 0xFFFFFFu) };
    uint32_t key[2] = { (uint32_t)seed, (uint32_t)(seed >> 32) };
    orc_philox4x32_10(ctr, key, out);
}

/* 53-bit uniform on [0,1) from two words. */
double orc_uniform53(uint32_t a, uint32_t b)
{
    return ((double)(a >> 5) * 67108864.0 + (double)(b >> 6)) * (1.0 / 9007199254740992.0);
}

/* Box-Muller pair from two uniforms; 1-u keeps the logarithm finite. */
void orc_normal2(uint32_t w[4], double* n0, double* n1)
{
    double u1 = orc_uniform53(w[0], w[1]);
    double u2 = orc_uniform53(w[2], w[3]);
    double rad = sqrt(-2.0 * log(1.0 - u1));
    *n0 = rad * cos(ORC_TWO_PI * u2);
    *n1 = rad * sin(ORC_TWO_PI * u2);
}

/* Integer choice in [0, n) from one word: floor(w * n / 2^32). */
static uint32_t orc_choose(uint32_t w, uint32_t n)
{
    return (uint32_t)(((uint64_t)w * (uint64_t)n) >> 32);
}

/* =================================================== HCT descreening term */
/* h(r; rt, s): contribution of a sphere of radius s at distance r to the
 * descreening integral of an atom of offset radius rt, as the closed form of
 * twice the integral over shells t of (fraction of the shell inside the
 * sphere) / t^2, for t from max(rt, |r-s|) to r+s, plus the fully-covered
 * shells from rt to s-r when the sphere engulfs the atom. */
double orc_hct(double r, double rt, double s)
{
    if (r == 0.0)                       /* concentric: only whole shells */
        return rt >= s ? 0.0 : 2.0 * (1.0 / rt - 1.0 / s);
    if (r + s <= rt)                    /* sphere lies inside the atom    */
        return 0.0;
    double L = fmax(rt, fabs(r - s));
    double U = r + s;
    double h = 1.0 / L - 1.0 / U
             + 0.25 * r * (1.0 / (U * U) - 1.0 / (L * L))
             + 0.5 / r * log(L / U)
             + 0.25 * s * s / r * (1.0 / (L * L) - 1.0 / (U * U));
    if (rt < s - r)                     /* atom engulfed by the sphere    */
        h += 2.0 * (1.0 / rt - 1.0 / L);
    return h;
}

/* Partial derivatives of orc_hct with respect to r, rt and s, obtained by
 * differentiating the closed form term by term with dU/dr = dU/ds = 1 and
 * dL/dx = 0 when L = rt, otherwise dL/dr = sign(r - s), dL/ds = sign(s - r)
 * (and dL/drt = 1 when L = rt). */
void orc_hct_grad(double r, double rt, double s, double* d_r, double* d_rt, double* d_s)
{
    *d_r = 0.0; *d_rt = 0.0; *d_s = 0.0;
    if (r == 0.0 || r + s <= rt) return;
    int L_is_rt = rt >= fabs(r - s);
    double L = L_is_rt ? rt : fabs(r - s);
    double U = r + s;
    double Lr  = L_is_rt ? 0.0 : (r > s ? 1.0 : -1.0);
    double Ls  = L_is_rt ? 0.0 : (s > r ? 1.0 : -1.0);
    double Lrt = L_is_rt ? 1.0 : 0.0;
    double iL = 1.0 / L, iU = 1.0 / U;
    double iL2 = iL * iL, iU2 = iU * iU, iL3 = iL2 * iL, iU3 = iU2 * iU;
    double lg = log(L / U);
    int engulfed = rt < s - r;

    /* d/dr */
    double dr = -Lr * iL2 + iU2
              + 0.25 * (iU2 - iL2)
              + 0.25 * r * (-2.0 * iU3 + 2.0 * Lr * iL3)
              - 0.5 / (r * r) * lg
              + 0.5 / r * (Lr * iL - iU)
              - 0.25 * s * s / (r * r) * (iL2 - iU2)
              + 0.25 * s * s / r * (-2.0 * Lr * iL3 + 2.0 * iU3);
    if (engulfed) dr += 2.0 * Lr * iL2;

    /* d/ds */
    double ds = -Ls * iL2 + iU2
              + 0.25 * r * (-2.0 * iU3 + 2.0 * Ls * iL3)
              + 0.5 / r * (Ls * iL - iU)
              + 0.5 * s / r * (iL2 - iU2)
              + 0.25 * s * s / r * (-2.0 * Ls * iL3 + 2.0 * iU3);
    if (engulfed) ds += 2.0 * Ls * iL2;

    /* d/drt */
    double drt = -Lrt * iL2
               + 0.25 * r * (2.0 * Lrt * iL3)
               + 0.5 / r * (Lrt * iL)
               + 0.25 * s * s / r * (-2.0 * Lrt * iL3);
    if (engulfed) drt += 2.0 * (-1.0 / (rt * rt) + Lrt * iL2);

    *d_r = dr; *d_s = ds; *d_rt = drt;
}

/* ============================================================ helpers */
static double orc_dist(const double* xyz, int i, int j, double d[3])
{
    d[0] = xyz[3 * i + 0] - xyz[3 * j + 0];
    d[1] = xyz[3 * i + 1] - xyz[3 * j + 1];
    d[2] = xyz[3 * i + 2] - xyz[3 * j + 2];
    return sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
}

/* GB screening function: a GB pair term is -k_e q_i q_j g(f_ij) and a self
 * term -(1/2) k_e q_i^2 g(R_i), with g(f) = (1/eps_in - exp(-kappa f)/eps_out)/f
 * (the solvent's dielectric response screened by salt; kappa = 0 gives tau/f,
 * tau = 1/eps_in - 1/eps_out). */
static double orc_g(const orc_gb* p, double f)
{
    return (1.0 / p->eps_in - exp(-p->kappa * f) / p->eps_out) / f;
}

/* dg/df */
static double orc_dg(const orc_gb* p, double f)
{
    double es = exp(-p->kappa * f);
    return -(1.0 / p->eps_in - es / p->eps_out) / (f * f) + p->kappa * es / (p->eps_out * f);
}

/* Pair cutoffs: a pair at distance r takes part in the pair energies (Coulomb,
 * GB, LJ) when r < cut, and in the descreening sum when r < rgbmax; a cutoff
 * of 0 means none.  Self terms are always present. */
static int orc_in_cut(const orc_gb* p, double r) { return p->cut <= 0.0 || r < p->cut; }
static int orc_in_rgb(const orc_gb* p, double r) { return p->rgbmax <= 0.0 || r < p->rgbmax; }

/* ====================================================== effective Born radii */
/* psi_i = rho~_i * (1/2) sum_{j != i} h(r_ij; rho~_i, S_j rho~_j);
 * 1/R_i = 1/rho~_i - tanh(alpha psi - beta psi^2 + gamma psi^3) / rho_i;
 * dR_i/dpsi_i = R_i^2 (1 - tanh^2) (alpha - 2 beta psi + 3 gamma psi^2) / rho_i. */
void orc_born(int n, const double* xyz, const double* rho, const double* scr,
              const orc_gb* p, double* psi, double* R, double* dRdpsi)
{
    #pragma omp parallel for schedule(dynamic, 8)
    for (int i = 0; i < n; ++i) {
        double rti = rho[i] - p->offset;
        double sum = 0.0;
        for (int j = 0; j < n; ++j) {
            if (j == i) continue;
            double d[3];
            double r = orc_dist(xyz, i, j, d);
            if (!orc_in_rgb(p, r)) continue;
            double sj = scr[j] * (rho[j] - p->offset);
            sum += orc_hct(r, rti, sj);
        }
        double ps = rti * 0.5 * sum;
        double phi = p->alpha * ps - p->beta * ps * ps + p->gamma * ps * ps * ps;
        double th = tanh(phi);
        double invR = 1.0 / rti - th / rho[i];
        double Ri = 1.0 / invR;
        if (psi) psi[i] = ps;
        R[i] = Ri;
        if (dRdpsi)
            dRdpsi[i] = Ri * Ri * (1.0 - th * th)
                      * (p->alpha - 2.0 * p->beta * ps + 3.0 * p->gamma * ps * ps) / rho[i];
    }
}

/* ============================================================== energies */
/* Still's pair function f = sqrt(r^2 + Ri Rj exp(-r^2 / (4 Ri Rj))). */
static double orc_fgb(double r, double Ri, double Rj)
{
    return sqrt(r * r + Ri * Rj * exp(-r * r / (4.0 * Ri * Rj)));
}

/* E[0] = E_GB (pairs i<j and the self terms), E[1] = E_Coulomb, E[2] = E_LJ,
 * all pairs within the cutoff, no exclusions; Lorentz-Berthelot LJ
 * combination. */
void orc_energy(int n, const double* xyz, const double* q, const double* R,
                const double* sig, const double* eps, const orc_gb* p, double E[3])
{
    double* row = (double*)calloc((size_t)3 * n, sizeof(double));
    #pragma omp parallel for schedule(dynamic, 8)
    for (int i = 0; i < n; ++i) {
        double egb = -0.5 * p->k_e * q[i] * q[i] * orc_g(p, R[i]);
        double ec = 0.0, elj = 0.0;
        for (int j = i + 1; j < n; ++j) {
            double d[3];
            double r = orc_dist(xyz, i, j, d);
            if (!orc_in_cut(p, r)) continue;
            double f = orc_fgb(r, R[i], R[j]);
            egb += -p->k_e * q[i] * q[j] * orc_g(p, f);
            ec  += p->k_e / p->eps_in * q[i] * q[j] / r;
            double sij = 0.5 * (sig[i] + sig[j]);
            double eij = sqrt(eps[i] * eps[j]);
            double sr6 = pow(sij / r, 6.0);
            elj += 4.0 * eij * (sr6 * sr6 - sr6);
        }
        row[3 * i] = egb; row[3 * i + 1] = ec; row[3 * i + 2] = elj;
    }
    E[0] = E[1] = E[2] = 0.0;
    for (int i = 0; i < n; ++i) { E[0] += row[3 * i]; E[1] += row[3 * i + 1]; E[2] += row[3 * i + 2]; }
    free(row);
}

/* Electrostatic energy E_C + E_GB at fixed Born radii (what a titration
 * attempt changes). */
double orc_elec_energy(int n, const double* xyz, const double* q, const double* R, const orc_gb* p)
{
    double* row = (double*)calloc((size_t)n, sizeof(double));
    #pragma omp parallel for schedule(dynamic, 8)
    for (int i = 0; i < n; ++i) {
        double e = -0.5 * p->k_e * q[i] * q[i] * orc_g(p, R[i]);
        for (int j = i + 1; j < n; ++j) {
            double d[3];
            double r = orc_dist(xyz, i, j, d);
            if (!orc_in_cut(p, r)) continue;
            double f = orc_fgb(r, R[i], R[j]);
            e += -p->k_e * q[i] * q[j] * orc_g(p, f) + p->k_e / p->eps_in * q[i] * q[j] / r;
        }
        row[i] = e;
    }
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += row[i];
    free(row);
    return s;
}

/* The symmetric electrostatic kernel: E_elec = (1/2) q^T K q with
 * K_ij = k_e (1/(eps_in r) - g(f_ij)) for i != j within the cutoff (0 beyond)
 * and K_ii = -k_e g(R_i). */
static double orc_K(int n, const double* xyz, const double* R, const orc_gb* p, int i, int j)
{
    (void)n;
    if (i == j) return -p->k_e * orc_g(p, R[i]);
    double d[3];
    double r = orc_dist(xyz, i, j, d);
    if (!orc_in_cut(p, r)) return 0.0;
    return p->k_e * (1.0 / (p->eps_in * r) - orc_g(p, orc_fgb(r, R[i], R[j])));
}

/* Titration energy change, plain definition: E_elec(q') - E_elec(q) with q'
 * equal to q except q'[idx[k]] = qnew[k]. */
double orc_delta_e_plain(int n, const double* xyz, const double* q, const double* R,
                         const orc_gb* p, int m, const int* idx, const double* qnew)
{
    double* q2 = (double*)malloc((size_t)n * sizeof(double));
    memcpy(q2, q, (size_t)n * sizeof(double));
    for (int k = 0; k < m; ++k) q2[idx[k]] = qnew[k];
    double e1 = orc_elec_energy(n, xyz, q2, R, p);
    double e0 = orc_elec_energy(n, xyz, q, R, p);
    free(q2);
    return e1 - e0;
}

/* Titration energy change, incremental form: with delta = q' - q supported on
 * the site, dE = sum_k delta_k (K q)_k + (1/2) sum_{k,l} delta_k delta_l K_kl. */
double orc_delta_e_incr(int n, const double* xyz, const double* q, const double* R,
                        const orc_gb* p, int m, const int* idx, const double* qnew)
{
    double lin = 0.0, quad = 0.0;
    for (int k = 0; k < m; ++k) {
        int a = idx[k];
        double dk = qnew[k] - q[a];
        double Kq = 0.0;
        for (int j = 0; j < n; ++j) Kq += orc_K(n, xyz, R, p, a, j) * q[j];
        lin += dk * Kq;
        for (int l = 0; l < m; ++l) {
            int b = idx[l];
            quad += dk * (qnew[l] - q[b]) * orc_K(n, xyz, R, p, a, b);
        }
    }
    return lin + 0.5 * quad;
}

/* Error scale of the incremental form (not a result of the method): the sum
 * of the absolute values of its terms,
 *   sum_k |delta_k| sum_j |K_kj q_j| + (1/2) sum_{k,l} |delta_k delta_l K_kl|.
 * An evaluation that rounds each term to relative precision u and adds them
 * up is off by at most a few u times this sum, however much the terms cancel. */
double orc_delta_e_abs(int n, const double* xyz, const double* q, const double* R,
                       const orc_gb* p, int m, const int* idx, const double* qnew)
{
    double lin = 0.0, quad = 0.0;
    for (int k = 0; k < m; ++k) {
        int a = idx[k];
        double dk = fabs(qnew[k] - q[a]);
        double Kq = 0.0;
        for (int j = 0; j < n; ++j) Kq += fabs(orc_K(n, xyz, R, p, a, j) * q[j]);
        lin += dk * Kq;
        for (int l = 0; l < m; ++l) {
            int b = idx[l];
            quad += fabs(dk * (qnew[l] - q[b]) * orc_K(n, xyz, R, p, a, b));
        }
    }
    return lin + 0.5 * quad;
}

/* ============================================================== gradients */
/* Analytic gradient of E = E_GB + E_C + E_LJ with respect to positions,
 * charges and intrinsic radii, by the chain rule through the Born radii:
 *   dE/dx_i = sum_j [dE_pair/dr_ij + c_i h_r(r_ij; rt_i, s_j) + c_j h_r(r_ij; rt_j, s_i)] (x_i - x_j)/r_ij
 *   c_i     = (dE/dR_i) (dR_i/dpsi_i) (rt_i / 2)
 *   dE/dq_i = sum_j K_ij q_j (self included)
 *   dE/drho_i = dE/dR_i [dR_i/drho_i at fixed psi + dR_i/dpsi_i (I_i + (rt_i/2) sum_j h_rt(r_ij; rt_i, s_j))]
 *             + S_i sum_{k != i} c_k h_s(r_ki; rt_k, s_i)
 * where I_i = (1/2) sum_j h(r_ij; rt_i, s_j), and h_r, h_rt, h_s are the partial derivatives of h.
 * Outputs: E[3] as orc_energy; dEdx AoS [3n]; dEdq [n]; dEdrho [n] (each may be NULL). */
void orc_gradient(int n, const double* xyz, const double* q, const double* rho, const double* scr,
                  const double* sig, const double* eps, const orc_gb* p,
                  double E[3], double* dEdx, double* dEdq, double* dEdrho)
{
    double* psi = (double*)malloc((size_t)n * sizeof(double));
    double* R = (double*)malloc((size_t)n * sizeof(double));
    double* dRdpsi = (double*)malloc((size_t)n * sizeof(double));
    double* dEdR = (double*)malloc((size_t)n * sizeof(double));
    double* c = (double*)malloc((size_t)n * sizeof(double));
    orc_born(n, xyz, rho, scr, p, psi, R, dRdpsi);
    if (E) orc_energy(n, xyz, q, R, sig, eps, p, E);

    /* dE/dR_i: self term plus every GB pair containing i. */
    #pragma omp parallel for schedule(dynamic, 8)
    for (int i = 0; i < n; ++i) {
        double g = -0.5 * p->k_e * q[i] * q[i] * orc_dg(p, R[i]);
        for (int j = 0; j < n; ++j) {
            if (j == i) continue;
            double d[3];
            double r = orc_dist(xyz, i, j, d);
            if (!orc_in_cut(p, r)) continue;
            double RR = R[i] * R[j];
            double D = r * r / (4.0 * RR);
            double f = orc_fgb(r, R[i], R[j]);
            double dfdRi = R[j] * exp(-D) * (1.0 + D) / (2.0 * f);
            g += -p->k_e * q[i] * q[j] * orc_dg(p, f) * dfdRi;
        }
        dEdR[i] = g;
        c[i] = g * dRdpsi[i] * 0.5 * (rho[i] - p->offset);
    }

    #pragma omp parallel for schedule(dynamic, 8)
    for (int i = 0; i < n; ++i) {
        double rti = rho[i] - p->offset;
        double si = scr[i] * rti;
        double gx = 0.0, gy = 0.0, gz = 0.0, gq = -p->k_e * q[i] * orc_g(p, R[i]);
        double sum_h = 0.0, sum_hrt = 0.0, sum_hs = 0.0;
        for (int j = 0; j < n; ++j) {
            if (j == i) continue;
            double d[3];
            double r = orc_dist(xyz, i, j, d);
            double rtj = rho[j] - p->offset;
            double sj = scr[j] * rtj;
            double dgb = 0.0, dc = 0.0, dlj = 0.0, dchain = 0.0;
            if (orc_in_cut(p, r)) {
                double RR = R[i] * R[j];
                double D = r * r / (4.0 * RR);
                double f = orc_fgb(r, R[i], R[j]);
                double dfdr = r / f * (1.0 - 0.25 * exp(-D));
                /* pair energy derivative with respect to r at fixed Born radii */
                dgb = -p->k_e * q[i] * q[j] * orc_dg(p, f) * dfdr;
                dc = -p->k_e / p->eps_in * q[i] * q[j] / (r * r);
                double sij = 0.5 * (sig[i] + sig[j]);
                double eij = sqrt(eps[i] * eps[j]);
                double sr6 = pow(sij / r, 6.0);
                dlj = 4.0 * eij * (-12.0 * sr6 * sr6 + 6.0 * sr6) / r;
                gq += (p->k_e * (1.0 / (p->eps_in * r) - orc_g(p, f))) * q[j];
            }
            if (orc_in_rgb(p, r)) {
                /* Born-radius chain terms through psi_i and psi_j */
                double hij_r, hij_rt, hij_s, hji_r, hji_rt, hji_s;
                orc_hct_grad(r, rti, sj, &hij_r, &hij_rt, &hij_s);
                orc_hct_grad(r, rtj, si, &hji_r, &hji_rt, &hji_s);
                dchain = c[i] * hij_r + c[j] * hji_r;
                sum_h += orc_hct(r, rti, sj);
                sum_hrt += hij_rt;
                sum_hs += c[j] * hji_s;
            }
            double g = (dgb + dc + dlj + dchain) / r;
            gx += g * d[0]; gy += g * d[1]; gz += g * d[2];
        }
        if (dEdx) { dEdx[3 * i] = gx; dEdx[3 * i + 1] = gy; dEdx[3 * i + 2] = gz; }
        if (dEdq) dEdq[i] = gq;
        if (dEdrho) {
            double ps = psi[i];
            double phi = p->alpha * ps - p->beta * ps * ps + p->gamma * ps * ps * ps;
            double th = tanh(phi);
            /* 1/R = 1/rt - tanh(phi)/rho: explicit dependence on rho through rt and rho */
            double dRdrho_fixed = R[i] * R[i] * (1.0 / (rti * rti) - th / (rho[i] * rho[i]));
            double I = 0.5 * sum_h;
            double dpsidrho = I + 0.5 * rti * sum_hrt;
            dEdrho[i] = dEdR[i] * (dRdrho_fixed + dRdpsi[i] * dpsidrho) + scr[i] * sum_hs;
        }
    }
    free(psi); free(R); free(dRdpsi); free(dEdR); free(c);
}

/* Harmonic tether E = k sum |x - x0|^2 and its gradient (added into dEdx). */
double orc_tether(int n, const double* xyz, const double* x0, double k, double* dEdx)
{
    double e = 0.0;
    for (int i = 0; i < 3 * n; ++i) {
        double d = xyz[i] - x0[i];
        e += k * d * d;
        if (dEdx) dEdx[i] += 2.0 * k * d;
    }
    return e;
}

/* =========================================================== batched E+F */
/* Loops the single-system functions over replicas laid out back to back
 * (replica r owns atoms atom_off[r] .. atom_off[r+1]-1).
 * E is [n_rep*3]; per-atom outputs may be NULL. */
void orc_eval_batch(int n_rep, const int* atom_off, const double* xyz, const double* q,
                    const double* rho, const double* scr, const double* sig, const double* eps,
                    const orc_gb* p, double* E, double* dEdx, double* dEdq, double* dEdrho)
{
    for (int r = 0; r < n_rep; ++r) {
        int a0 = atom_off[r], n = atom_off[r + 1] - a0;
        orc_gradient(n, xyz + 3 * a0, q + a0, rho + a0, scr + a0, sig + a0, eps + a0, p,
                     E ? E + 3 * r : NULL, dEdx ? dEdx + 3 * a0 : NULL,
                     dEdq ? dEdq + a0 : NULL, dEdrho ? dEdrho + a0 : NULL);
    }
}

void orc_born_batch(int n_rep, const int* atom_off, const double* xyz, const double* rho,
                    const double* scr, const orc_gb* p, double* psi, double* R, double* dRdpsi)
{
    for (int r = 0; r < n_rep; ++r) {
        int a0 = atom_off[r], n = atom_off[r + 1] - a0;
        orc_born(n, xyz + 3 * a0, rho + a0, scr + a0, p, psi ? psi + a0 : NULL, R + a0,
                 dRdpsi ? dRdpsi + a0 : NULL);
    }
}

/* ======================================================= MD / MC / REMD */
typedef struct {
    /* layout */
    int n_rep;
    const int* atom_off;
    /* titratable sites; replica r owns sites rep_site_off[r] .. rep_site_off[r+1]-1 */
    int n_sites, max_states;
    const int* rep_site_off;
    const int* site_off;       /* site s owns site_atoms[site_off[s] .. site_off[s+1]-1] */
    const int* site_atoms;     /* flat atom index */
    const int* site_type;      /* 0 = pH, 1 = redox */
    const int* n_states;
    const double* state_q;     /* [slot * max_states + state] */
    const int* state_nH;       /* [site * max_states + state] */
    const int* state_ne;
    const double* G_ref;       /* [site * max_states + state], kcal/mol */
    const double* ref_value;   /* pKa_ref (pH sites) or E0_ref in V (redox sites) */
    /* replica grid: n_inst independent grids of nE x npH x nT x nHam points,
     * grid point g = ((iE * npH + ipH) * nT + iT) * nHam + iH; H_scale[iH] is
     * the scale l of the GB + Coulomb + LJ energy at Hamiltonian level iH */
    int n_inst, nE, npH, nT, nHam;
    const double* E_vals; const double* pH_vals; const double* T_vals; const double* H_scale;
    int n_dims; int dim_order[4];
    /* per-atom parameters */
    const double* rho; const double* scr; const double* sig; const double* eps;
    const double* mass; const double* x0;
    orc_gb gb;
    double k_tether, dt, gamma_ps;
    int mc_every, ex_every, eps_mode;   /* eps_mode 0: semi-grand energy; 1: potential U */
    uint64_t seed;
} orc_md_cfg;

typedef struct {
    double* xyz;            /* AoS [3 Ntot] */
    double* v;              /* AoS [3 Ntot] */
    double* q;              /* [Ntot] */
    double* F;              /* AoS [3 Ntot], forces of U_l at xyz (tether included) */
    double* E;              /* [n_rep * 4]: GB, Coulomb, LJ (unscaled), tether at xyz */
    int* site_state;        /* [n_sites] */
    int* target_idx;        /* [n_rep * 4]: iE, ipH, iT, iH */
    int* grid_rep;          /* [n_inst * nE * npH * nT * nHam] */
    long long* mc_att;      /* [n_sites] */
    long long* mc_acc;
    long long* ex_att;      /* [4 * n_inst * G], indexed dim * (n_inst G) + global lower point */
    long long* ex_acc;
} orc_md_state;

/* Scale l of replica r's GB + Coulomb + LJ energy (its Hamiltonian level). */
static double orc_lambda(const orc_md_cfg* c, const int* target_idx, int r)
{
    return c->H_scale ? c->H_scale[target_idx[ORC_NDIM * r + ORC_DIM_H]] : 1.0;
}

/* Forces of U_l = l (E_GB + E_C + E_LJ) + E_tether for replica r at its
 * positions; the energy components are stored unscaled. */
static void orc_forces_one(const orc_md_cfg* c, orc_md_state* s, int r)
{
    int a0 = c->atom_off[r], n = c->atom_off[r + 1] - a0;
    double* g = (double*)calloc((size_t)3 * n, sizeof(double));
    double E3[3];
    orc_gradient(n, s->xyz + 3 * a0, s->q + a0, c->rho + a0, c->scr + a0, c->sig + a0, c->eps + a0,
                 &c->gb, E3, g, NULL, NULL);
    double lam = orc_lambda(c, s->target_idx, r);
    for (int i = 0; i < 3 * n; ++i) g[i] *= lam;
    double et = orc_tether(n, s->xyz + 3 * a0, c->x0 + 3 * a0, c->k_tether, g);
    for (int i = 0; i < 3 * n; ++i) s->F[3 * a0 + i] = -g[i];
    s->E[4 * r + 0] = E3[0]; s->E[4 * r + 1] = E3[1]; s->E[4 * r + 2] = E3[2]; s->E[4 * r + 3] = et;
    free(g);
}

/* One Monte Carlo attempt on one site type for replica r (eqs. 1-2 weights):
 *   dG = l dE_elec - [G_ref(s') - G_ref(s)] + kT ln10 (pH - pKa_ref) (N_H(s') - N_H(s))   (pH site)
 *   dG = l dE_elec - [G_ref(s') - G_ref(s)] + F (E - E0_ref) (N_e(s') - N_e(s))           (redox site)
 * (l: the replica's Hamiltonian scale, which multiplies its electrostatic
 * energy) accepted iff dG <= 0 or u < exp(-dG / kT). Born radii are those of
 * the current geometry. */
static void orc_mc_one(const orc_md_cfg* c, orc_md_state* s, int r, const double* R,
                       uint64_t step, int type)
{
    int s0 = c->rep_site_off[r], s1 = c->rep_site_off[r + 1];
    int cnt = 0;
    for (int k = s0; k < s1; ++k) cnt += c->site_type[k] == type;
    if (cnt == 0) return;
    uint32_t w[4];
    orc_draw(c->seed, 0u, (uint32_t)r, step, type == 0 ? ORC_STREAM_MCPH : ORC_STREAM_MCRED, w);
    uint32_t pick = orc_choose(w[0], (uint32_t)cnt);
    int site = -1;
    for (int k = s0, m = 0; k < s1; ++k) {
        if (c->site_type[k] != type) continue;
        if ((uint32_t)m == pick) { site = k; break; }
        ++m;
    }
    int ms = c->max_states;
    int cur = s->site_state[site];
    uint32_t off = orc_choose(w[1], (uint32_t)(c->n_states[site] - 1));
    int nw = (int)off < cur ? (int)off : (int)off + 1;

    int a0 = c->atom_off[r], n = c->atom_off[r + 1] - a0;
    int m = c->site_off[site + 1] - c->site_off[site];
    int* idx = (int*)malloc((size_t)m * sizeof(int));
    double* qn = (double*)malloc((size_t)m * sizeof(double));
    for (int k = 0; k < m; ++k) {
        int slot = c->site_off[site] + k;
        idx[k] = c->site_atoms[slot] - a0;
        qn[k] = c->state_q[(size_t)slot * ms + nw];
    }
    double dE = orc_delta_e_plain(n, s->xyz + 3 * a0, s->q + a0, R, &c->gb, m, idx, qn);
    double T = c->T_vals[s->target_idx[ORC_NDIM * r + ORC_DIM_T]];
    double kT = ORC_KB * T;
    double dG = orc_lambda(c, s->target_idx, r) * dE - (c->G_ref[site * ms + nw] - c->G_ref[site * ms + cur]);
    if (type == 0) {
        double pH = c->pH_vals[s->target_idx[ORC_NDIM * r + ORC_DIM_PH]];
        dG += kT * ORC_LN10 * (pH - c->ref_value[site])
            * (double)(c->state_nH[site * ms + nw] - c->state_nH[site * ms + cur]);
    } else {
        double Ev = c->E_vals[s->target_idx[ORC_NDIM * r + ORC_DIM_E]];
        dG += ORC_FARAD * (Ev - c->ref_value[site])
            * (double)(c->state_ne[site * ms + nw] - c->state_ne[site * ms + cur]);
    }
    double u = orc_uniform53(w[2], w[3]);
    if (s->mc_att) s->mc_att[site] += 1;
    if (dG <= 0.0 || u < exp(-dG / kT)) {
        s->site_state[site] = nw;
        for (int k = 0; k < m; ++k) s->q[a0 + idx[k]] = qn[k];
        if (s->mc_acc) s->mc_acc[site] += 1;
    }
    free(idx); free(qn);
}

/* Protons, electrons and the exchange energy of replica r.  eps_mode 0 is the
 * energy whose Boltzmann factor the titration moves sample at fixed pH and E:
 * U - sum G_ref(s) + sum_redox F (E - E0_ref) N_e(s)  (the pH term carries kT
 * and cancels in eq. 5); eps_mode 1 is the potential energy U alone.  U is
 * the replica's own potential U_l = l (E_GB + E_C + E_LJ) + E_tether. */
void orc_replica_counts(const orc_md_cfg* c, const int* site_state, const int* target_idx,
                        const double* E4, int r, int* nH, int* ne, double* epsT)
{
    int ms = c->max_states;
    int h = 0, e = 0;
    double U = orc_lambda(c, target_idx, r) * (E4[4 * r] + E4[4 * r + 1] + E4[4 * r + 2]) + E4[4 * r + 3];
    double extra = 0.0;
    double Ev = c->E_vals[target_idx[ORC_NDIM * r + ORC_DIM_E]];
    for (int k = c->rep_site_off[r]; k < c->rep_site_off[r + 1]; ++k) {
        int st = site_state[k];
        h += c->state_nH[k * ms + st];
        e += c->state_ne[k * ms + st];
        extra -= c->G_ref[k * ms + st];
        if (c->site_type[k] == 1)
            extra += ORC_FARAD * (Ev - c->ref_value[k]) * (double)c->state_ne[k * ms + st];
    }
    *nH = h; *ne = e;
    *epsT = c->eps_mode == 0 ? U + extra : U;
}

/* Potential energy of a configuration whose energy components (GB, Coulomb,
 * LJ, tether) are E4[0..3], under the Hamiltonian of scale l. */
static double orc_U(double l, const double* E4)
{
    return l * (E4[0] + E4[1] + E4[2]) + E4[3];
}

/* One exchange attempt (attempt index a): dimension dim_order[a % n_dims],
 * parity (a / n_dims) % 2; pairs of grid points (k, k+1) along that dimension
 * with k of that parity, within each line of equal other targets; acceptance
 * eq. 3, 4 or 5 against u drawn for the lower grid point.  A Hamiltonian
 * attempt between replica i (level k) and j (level k+1) at temperature T
 * accepts with min(1, exp(-[U_k(x_j) + U_k+1(x_i) - U_k(x_i) - U_k+1(x_j)] / kT)),
 * the energies formed from the replicas' components E4 [n_rep * 4].  On
 * acceptance the two replicas swap their target index in that dimension; a
 * temperature swap scales each replica's velocities by sqrt(T_new / T_old):
 * the factor is multiplied into vscale[replica] (vscale may be NULL). */
void orc_exchange(const orc_md_cfg* c, long long a, const int* nH, const int* ne, const double* epsT,
                  const double* E4, int* target_idx, int* grid_rep, double* vscale,
                  long long* ex_att, long long* ex_acc)
{
    int d = c->dim_order[a % c->n_dims];
    int parity = (int)((a / c->n_dims) % 2);
    int dimsz[ORC_NDIM] = { c->nE, c->npH, c->nT, c->nHam };
    int G = c->nE * c->npH * c->nT * c->nHam;
    int GT = G * c->n_inst;
    for (int inst = 0; inst < c->n_inst; ++inst) {
        for (int g = 0; g < G; ++g) {
            int iH = g % c->nHam, iT = (g / c->nHam) % c->nT;
            int ipH = (g / (c->nHam * c->nT)) % c->npH, iE = g / (c->nHam * c->nT * c->npH);
            int coord[ORC_NDIM] = { iE, ipH, iT, iH };
            int k = coord[d];
            if (k % 2 != parity || k + 1 >= dimsz[d]) continue;
            int c2[ORC_NDIM] = { iE, ipH, iT, iH };
            c2[d] = k + 1;
            int g2 = ((c2[0] * c->npH + c2[1]) * c->nT + c2[2]) * c->nHam + c2[3];
            int gl = inst * G + g, gu = inst * G + g2;
            int ri = grid_rep[gl], rj = grid_rep[gu];
            double delta;
            if (d == ORC_DIM_PH) {
                delta = ORC_LN10 * (c->pH_vals[k] - c->pH_vals[k + 1]) * (double)(nH[ri] - nH[rj]);
            } else if (d == ORC_DIM_E) {
                double kT = ORC_KB * c->T_vals[iT];
                delta = ORC_FARAD / kT * (c->E_vals[k] - c->E_vals[k + 1]) * (double)(ne[ri] - ne[rj]);
            } else if (d == ORC_DIM_T) {
                double bi = 1.0 / (ORC_KB * c->T_vals[k]), bj = 1.0 / (ORC_KB * c->T_vals[k + 1]);
                delta = (bi - bj) * (epsT[ri] - epsT[rj]);
            } else {
                double kT = ORC_KB * c->T_vals[iT];
                double lk = c->H_scale[k], lk1 = c->H_scale[k + 1];
                const double* Ei = E4 + 4 * ri;
                const double* Ej = E4 + 4 * rj;
                delta = -((orc_U(lk, Ej) + orc_U(lk1, Ei)) - (orc_U(lk, Ei) + orc_U(lk1, Ej))) / kT;
            }
            uint32_t w[4];
            orc_draw(c->seed, 0u, (uint32_t)gl, (uint64_t)a, ORC_STREAM_EX, w);
            double u = orc_uniform53(w[0], w[1]);
            if (ex_att) ex_att[(size_t)d * GT + gl] += 1;
            if (delta >= 0.0 || u < exp(delta)) {
                target_idx[ORC_NDIM * ri + d] = k + 1;
                target_idx[ORC_NDIM * rj + d] = k;
                grid_rep[gl] = rj; grid_rep[gu] = ri;
                if (ex_acc) ex_acc[(size_t)d * GT + gl] += 1;
                if (d == ORC_DIM_T && vscale) {
                    vscale[ri] *= sqrt(c->T_vals[k + 1] / c->T_vals[k]);
                    vscale[rj] *= sqrt(c->T_vals[k] / c->T_vals[k + 1]);
                }
            }
        }
    }
}

/* Run n_steps BAOAB Langevin steps for every replica (step indices step0 ..
 * step0 + n_steps - 1).  Step n: half kick with F_n, half drift, exact
 * Ornstein-Uhlenbeck velocity update at the replica's temperature, half
 * drift; if (n+1) % mc_every == 0 a protonation then a redox attempt at the
 * new positions; forces at the new positions; half kick; then if
 * (n+1) % ex_every == 0 exchange attempt (n+1)/ex_every - 1.
 * With init_forces set, forces and energies are first computed at xyz. */
int orc_md_run(const orc_md_cfg* c, orc_md_state* s, long long step0, int n_steps, int init_forces)
{
    int ntot = c->atom_off[c->n_rep];
    if (init_forces)
        for (int r = 0; r < c->n_rep; ++r) orc_forces_one(c, s, r);
    int* nH = (int*)malloc((size_t)c->n_rep * sizeof(int));
    int* ne = (int*)malloc((size_t)c->n_rep * sizeof(int));
    double* epsT = (double*)malloc((size_t)c->n_rep * sizeof(double));
    double* vscale = (double*)malloc((size_t)c->n_rep * sizeof(double));
    double* lam_old = (double*)malloc((size_t)c->n_rep * sizeof(double));
    double* R = (double*)malloc((size_t)ntot * sizeof(double));
    double c1 = exp(-c->gamma_ps * c->dt);
    double c2 = sqrt(1.0 - c1 * c1);
    double hdt = 0.5 * c->dt;
    for (int st = 0; st < n_steps; ++st) {
        uint64_t n = (uint64_t)(step0 + st);
        for (int r = 0; r < c->n_rep; ++r) {
            int a0 = c->atom_off[r], na = c->atom_off[r + 1] - a0;
            double kT = ORC_KB * c->T_vals[s->target_idx[ORC_NDIM * r + ORC_DIM_T]];
            for (int i = 0; i < na; ++i) {
                int a = a0 + i;
                double im = ORC_CONV / c->mass[a];
                double xi[4];
                uint32_t w[4];
                orc_draw(c->seed, (uint32_t)(2 * i), (uint32_t)r, n, ORC_STREAM_O, w);
                orc_normal2(w, &xi[0], &xi[1]);
                orc_draw(c->seed, (uint32_t)(2 * i + 1), (uint32_t)r, n, ORC_STREAM_O, w);
                orc_normal2(w, &xi[2], &xi[3]);
                double sd = sqrt(kT * im);
                for (int d = 0; d < 3; ++d) {
                    double* v = &s->v[3 * a + d];
                    double* x = &s->xyz[3 * a + d];
                    *v += hdt * s->F[3 * a + d] * im;
                    *x += hdt * *v;
                    *v = c1 * *v + c2 * sd * xi[d];
                    *x += hdt * *v;
                }
            }
            if (c->mc_every > 0 && (n + 1) % (uint64_t)c->mc_every == 0) {
                orc_born(na, s->xyz + 3 * a0, c->rho + a0, c->scr + a0, &c->gb, NULL, R + a0, NULL);
                orc_mc_one(c, s, r, R + a0, n, 0);
                orc_mc_one(c, s, r, R + a0, n, 1);
            }
            orc_forces_one(c, s, r);
            for (int i = 0; i < na; ++i) {
                int a = a0 + i;
                double im = ORC_CONV / c->mass[a];
                for (int d = 0; d < 3; ++d) s->v[3 * a + d] += hdt * s->F[3 * a + d] * im;
            }
        }
        if (c->ex_every > 0 && (n + 1) % (uint64_t)c->ex_every == 0) {
            long long att = (long long)((n + 1) / (uint64_t)c->ex_every) - 1;
            for (int r = 0; r < c->n_rep; ++r) {
                orc_replica_counts(c, s->site_state, s->target_idx, s->E, r, &nH[r], &ne[r], &epsT[r]);
                vscale[r] = 1.0;
                lam_old[r] = orc_lambda(c, s->target_idx, r);
            }
            orc_exchange(c, att, nH, ne, epsT, s->E, s->target_idx, s->grid_rep, vscale,
                         s->ex_att, s->ex_acc);
            for (int r = 0; r < c->n_rep; ++r) {
                /* a replica given another Hamiltonian needs that Hamiltonian's
                 * forces for the next half kick */
                if (orc_lambda(c, s->target_idx, r) != lam_old[r]) orc_forces_one(c, s, r);
                if (vscale[r] == 1.0) continue;
                for (int a = c->atom_off[r]; a < c->atom_off[r + 1]; ++a)
                    for (int d = 0; d < 3; ++d) s->v[3 * a + d] *= vscale[r];
            }
        }
    }
    free(nH); free(ne); free(epsT); free(vscale); free(lam_old); free(R);
    return 0;
}

/* Expose the constants so the tests can state what the oracle used. */
void orc_constants(double out[4])
{
    out[0] = ORC_KB; out[1] = ORC_FARAD; out[2] = ORC_LN10; out[3] = ORC_CONV;
}
