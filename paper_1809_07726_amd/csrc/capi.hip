// capi.hip -- the C ABI declared in include/gbremd.h: argument checks,
// context and workspace, the per-call launch sequences, kernel timing and the
// captured per-step graphs of md_step.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "gbr_internal.h"
#include "pair_list.h"

using namespace gbr;

namespace {

thread_local std::string g_last_error;

int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

int hip_fail(hipError_t e, const char* what) {
    return fail(GBR_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

#define GBR_HIP(call)                                          \
    do {                                                       \
        hipError_t e_ = (call);                                \
        if (e_ != hipSuccess) return hip_fail(e_, #call);      \
    } while (0)

template <typename T>
int dev_alloc(T** p, size_t n) {
    if (n == 0) n = 1;
    hipError_t e = hipMalloc(reinterpret_cast<void**>(p), n * sizeof(T));
    if (e != hipSuccess) return fail(GBR_E_NOMEM, "hipMalloc(%zu bytes): %s", n * sizeof(T),
                                     hipGetErrorString(e));
    return GBR_OK;
}

// Timing: a pair of events per timed launch when enabled.  ext: the launch
// records them itself, from its own dispatch (the pair kernels, through
// hipExtLaunchKernel: no marker packets between kernels); otherwise they are
// recorded on the stream around the launch.
struct Timed {
    gbr_ctx* c;
    int kind;
    hipStream_t s;
    bool ext;
    LaunchEvents ev;
    Timed(gbr_ctx* c_, int kind_, hipStream_t s_, bool ext_ = false) : c(c_), kind(kind_), s(s_), ext(ext_) {
        Timer& t = c->timer;
        if (!(t.mask & (1 << kind_))) return;
        if (t.used + 2 > t.pool.size()) {
            size_t old = t.pool.size();
            t.pool.resize(old + 512);
            for (size_t i = old; i < t.pool.size(); ++i)
                if (hipEventCreate(&t.pool[i]) != hipSuccess) t.pool[i] = nullptr;
        }
        hipEvent_t start = t.pool[t.used], stop = t.pool[t.used + 1];
        if (!start || !stop) return;
        t.kind.push_back(kind);
        t.used += 2;
        ev.start = start;
        ev.stop = stop;
        if (!ext) (void)hipEventRecord(start, s);
    }
    ~Timed() {
        if (ev.stop && !ext) (void)hipEventRecord(ev.stop, s);
    }
};

// The static scratch of gb_born_radii_noalloc: 64-bit fixed-point descreening
// sums of up to GBR_NOALLOC_MAX_ATOMS atoms, one copy per device.  Host code
// never passes `scratch` itself to a kernel (on the host it names a stand-in):
// it looks up the device address once per device and uses that.
static __device__ __align__(256) int64_t scratch[GBR_NOALLOC_MAX_ATOMS];

constexpr int MAX_DEVICES = 64;
struct NoallocDev {
    int64_t* scratch = nullptr;   // device address of `scratch` on that device
    int n_cu = 0;
};
std::mutex g_noalloc_mu;
NoallocDev g_noalloc[MAX_DEVICES];

// Device address of the scratch array on the current device dev (looked up
// on first use) and its CU count; checks that the device is gfx950.
int noalloc_device(int dev, NoallocDev* out) {
    if (dev < 0 || dev >= MAX_DEVICES) return fail(GBR_E_INVAL, "device %d out of range", dev);
    std::lock_guard<std::mutex> lk(g_noalloc_mu);
    NoallocDev& d = g_noalloc[dev];
    if (!d.scratch) {
        hipDeviceProp_t prop;
        GBR_HIP(hipGetDeviceProperties(&prop, dev));
        if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
            return fail(GBR_E_NODEVICE, "device %d is %s; this library is built for gfx950", dev,
                        prop.gcnArchName);
        void* p = nullptr;
        GBR_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        d.n_cu = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
        d.scratch = static_cast<int64_t*>(p);
    }
    *out = d;
    return GBR_OK;
}

int check_ctx(const gbr_ctx* c) {
    if (!c) return fail(GBR_E_INVAL, "null context");
    // launching on another device with this context's pointers would fault
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != c->device)
        return fail(GBR_E_INVAL, "the context belongs to device %d but device %d is current", c->device, dev);
    return GBR_OK;
}

#define REQ(p) \
    do { if (!(p)) return fail(GBR_E_INVAL, "%s: required pointer %s is null", __func__, #p); } while (0)

int check_sites(const gbr_ctx* c, const gbr_sites& s) {
    if (s.n_sites < 0) return fail(GBR_E_INVAL, "n_sites < 0");
    if (s.n_sites == 0) return GBR_OK;
    if (s.max_states < 2 || s.max_states > 8) return fail(GBR_E_INVAL, "max_states must be 2..8");
    if (!s.rep_site_off || !s.site_off || !s.site_atoms || !s.site_rep || !s.site_type ||
        !s.n_states || !s.state_q || !s.state_nH || !s.state_ne || !s.G_ref || !s.ref_value)
        return fail(GBR_E_INVAL, "gbr_sites: a table pointer is null");
    (void)c;
    return GBR_OK;
}

int check_grid(const gbr_ctx* c, const gbr_grid& g) {
    if (g.n_inst < 1 || g.nE < 1 || g.npH < 1 || g.nT < 1 || g.nHam < 1)
        return fail(GBR_E_INVAL, "grid sizes must be >= 1");
    const long long G = (long long)g.n_inst * g.nE * g.npH * g.nT * g.nHam;
    if (G != c->n_rep)
        return fail(GBR_E_INVAL, "grid n_inst*nE*npH*nT*nHam (%lld) != n_rep (%d)", G, c->n_rep);
    if (!g.E_vals || !g.pH_vals || !g.T_vals) return fail(GBR_E_INVAL, "grid value table is null");
    if (g.nHam > 1 && !g.H_scale) return fail(GBR_E_INVAL, "nHam > 1 needs H_scale");
    if (g.n_dims < 1 || g.n_dims > GBR_N_DIMS) return fail(GBR_E_INVAL, "n_dims must be 1..4");
    for (int k = 0; k < g.n_dims; ++k)
        if (g.dim_order[k] < 0 || g.dim_order[k] >= GBR_N_DIMS) return fail(GBR_E_INVAL, "bad dim_order");
    return GBR_OK;
}

int upload(void* dst, const void* src, size_t bytes) {
    GBR_HIP(hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice));
    return GBR_OK;
}

// One force evaluation inside md_step (the caller has cleared the accumulators);
// advance: the evaluation belongs to a step, whose counter then advances.
int md_forces(gbr_ctx* c, const MDArgs& a, bool with_mc, bool advance, hipStream_t s) {
    hipError_t e = launch_pack(c, a.st.xyz, s);
    if (e != hipSuccess) return hip_fail(e, "pack");
    {
        Timed t(c, GBR_K_BORN_PAIR, s, true);
        e = launch_born_pair(c, a.st.xyz, a.pr.rho, a.pr.screen, s, t.ev);
    }
    if (e != hipSuccess) return hip_fail(e, "born pair");
    {
        Timed t(c, GBR_K_PER_ATOM, s);
        e = launch_born_finalize(c, a.pr.rho, a.st.R, a.st.dRdpsi, nullptr, s);
    }
    if (e != hipSuccess) return hip_fail(e, "born finalize");
    if (with_mc) {
        Timed t(c, GBR_K_TITRATION, s);
        e = launch_mc(c, a, s);
        if (e != hipSuccess) return hip_fail(e, "mc");
    }
    {
        Timed t(c, GBR_K_ENERGY_PAIR, s, true);
        e = launch_energy_pair(c, a.st.xyz, a.st.q, a.st.R, a.pr.sigma, a.pr.eps, a.st.force_fx,
                               nullptr, s, t.ev);
    }
    if (e != hipSuccess) return hip_fail(e, "energy pair");
    {
        Timed t(c, GBR_K_PER_ATOM, s);
        e = launch_coef(c, a.st.q, a.pr.rho, a.st.R, a.st.dRdpsi, a.st.energy_fx, nullptr,
                        advance ? c->step : nullptr, s);
    }
    if (e != hipSuccess) return hip_fail(e, "coef");
    {
        Timed t(c, GBR_K_CHAIN_PAIR, s, true);
        e = launch_chain_pair(c, a.st.xyz, a.pr.rho, a.pr.screen, a.st.force_fx, nullptr, s, t.ev);
    }
    if (e != hipSuccess) return hip_fail(e, "chain pair");
    return GBR_OK;
}

// Step kinds: MC attempts, exchange attempt after the step, the step opens
// with the fused kernel that also closes the previous step, the step is closed
// by its own k_md_last (last step of the call, or an exchange follows).
enum { STEP_MC = 1, STEP_EX = 2, STEP_MID = 4, STEP_LAST = 8 };

// The launches of one MD step.
int md_one_step(gbr_ctx* c, const MDArgs& a, int kind, hipStream_t s) {
    hipError_t e;
    {
        Timed t(c, GBR_K_PER_ATOM, s);
        e = launch_md_first(c, a, (kind & STEP_MID) != 0, s);
    }
    if (e != hipSuccess) return hip_fail(e, "md first");
    int rc = md_forces(c, a, (kind & STEP_MC) != 0, true, s);
    if (rc) return rc;
    if (!(kind & STEP_LAST)) return GBR_OK;       // the next step's kernel closes this one
    {
        Timed t(c, GBR_K_PER_ATOM, s);
        e = launch_md_last(c, a, 1, s);
    }
    if (e != hipSuccess) return hip_fail(e, "md last");
    if (kind & STEP_EX) {
        Timed t(c, GBR_K_EXCHANGE, s);
        const bool ham = a.pr.grid.nHam > 1;
        e = launch_exchange_inputs(c, a.st, a.pr, c->ex_nH, c->ex_ne, c->ex_eps,
                                   ham ? c->ex_enb : nullptr, s);
        if (e == hipSuccess)
            e = launch_exchange(c, a.pr.grid, 0, c->step, a.pr.ex_every, c->ex_nH, c->ex_ne,
                                c->ex_eps, c->ex_enb, a.st.target_idx, a.st.grid_rep,
                                c->ex_vscale, ham ? c->ex_fscale : nullptr, a.st.ex_stats,
                                a.seed, s);
        if (e == hipSuccess)
            e = launch_apply_swaps(c, a, c->ex_vscale, ham ? c->ex_fscale : nullptr, s);
        if (e != hipSuccess) return hip_fail(e, "exchange");
    }
    return GBR_OK;
}

struct Fnv {
    uint64_t h = 1469598103934665603ull;
    template <typename T> void add(const T& v) {
        const unsigned char* p = reinterpret_cast<const unsigned char*>(&v);
        for (size_t i = 0; i < sizeof(T); ++i) { h ^= p[i]; h *= 1099511628211ull; }
    }
};

// Key of a captured step graph: every pointer and scalar the step's kernels take
// (field by field, so struct padding never enters the key).
uint64_t hash_args(const MDArgs& a) {
    Fnv f;
    const gbr_md_state& s = a.st;
    const gbr_md_params& p = a.pr;
    f.add(s.xyz); f.add(s.v); f.add(s.q); f.add(s.force_fx); f.add(s.energy_fx); f.add(s.R);
    f.add(s.dRdpsi); f.add(s.site_state); f.add(s.target_idx); f.add(s.grid_rep); f.add(s.ke);
    f.add(s.mc_stats); f.add(s.ex_stats);
    f.add(p.rho); f.add(p.screen); f.add(p.sigma); f.add(p.eps); f.add(p.mass); f.add(p.x0);
    f.add(p.k_tether); f.add(p.dt); f.add(p.gamma); f.add(p.mc_every); f.add(p.ex_every);
    f.add(p.eps_mode);
    const gbr_sites& t = p.sites;
    f.add(t.n_sites); f.add(t.max_states); f.add(t.rep_site_off); f.add(t.site_off);
    f.add(t.site_atoms); f.add(t.site_rep); f.add(t.site_type); f.add(t.n_states); f.add(t.state_q);
    f.add(t.state_nH); f.add(t.state_ne); f.add(t.G_ref); f.add(t.ref_value);
    const gbr_grid& g = p.grid;
    f.add(g.n_inst); f.add(g.nE); f.add(g.npH); f.add(g.nT); f.add(g.nHam); f.add(g.E_vals);
    f.add(g.pH_vals); f.add(g.T_vals); f.add(g.H_scale); f.add(g.n_dims);
    for (int k = 0; k < GBR_N_DIMS; ++k) f.add(g.dim_order[k]);
    f.add(a.seed);
    return f.h | 1ull;
}

// The pair work list of blocking index k (NI = 1, 2, 4, 8) at the context's
// split level, and with both cutoffs its packed parts; frees what an earlier
// build left.  The packed-list buffers (tile boxes, counters) must exist.
void free_list(gbr::PairList& L) {
    (void)hipFree(L.items); (void)hipFree(L.iblk); (void)hipFree(L.blk_p0); (void)hipFree(L.win);
    (void)hipFree(L.blk_win);
    L.items = nullptr; L.iblk = nullptr; L.blk_p0 = nullptr; L.win = nullptr; L.blk_win = nullptr;
    for (int v = 0; v < 2; ++v) {
        (void)hipFree(L.run[v]); (void)hipFree(L.blk_count[v]); (void)hipFree(L.pk_hdr[v]);
        (void)hipFree(L.pk_j[v]);
        L.run[v] = nullptr; L.blk_count[v] = nullptr; L.pk_hdr[v] = nullptr; L.pk_j[v] = nullptr;
    }
}

int build_list(gbr_ctx* c, int k) {
    static const int nis[4] = {1, 2, 4, 8};
    static_assert(sizeof(gbr::PairItem) == sizeof(int2), "item layout");
    static_assert(sizeof(gbr::PackWindow) == sizeof(int4), "window layout");
    gbr::PairList& L = c->lists[k];
    free_list(L);
    const int32_t n_rep = c->n_rep;
    std::vector<gbr::PairItem> items;
    gbr::build_pair_items(c->h_atom_off.data(), n_rep, nis[k], items, c->split_den);
    if (items.size() > 0x7FFFFFFF) return fail(GBR_E_INVAL, "work list too long");
    int rc = GBR_OK;
    L.ni = nis[k];
    L.n_items = (int32_t)items.size();
    if ((rc = dev_alloc(&L.items, items.size()))) return rc;
    if (!items.empty() && (rc = upload(L.items, items.data(), sizeof(int2) * items.size()))) return rc;
    if (!c->packed) return GBR_OK;
    std::vector<gbr::PairItem> intra, iblocks;
    std::vector<int32_t> p0, blk_win;
    std::vector<gbr::PackWindow> wins;
    int64_t cap = 0;
    gbr::build_packed_parts(c->h_atom_off.data(), n_rep, nis[k], items, intra, iblocks, p0, wins, blk_win, cap);
    if ((int64_t)intra.size() + cap > 0x7FFFFFFF || cap * 64 > 0x7FFFFFFF)
        return fail(GBR_E_INVAL, "work list too long");
    L.n_intra = (int32_t)intra.size();
    L.n_iblk = (int32_t)iblocks.size();
    L.n_win = (int32_t)wins.size();
    L.pk_cap = cap;
    if ((rc = dev_alloc(&L.iblk, iblocks.size()))) return rc;
    if (!iblocks.empty() && (rc = upload(L.iblk, iblocks.data(), sizeof(int2) * iblocks.size()))) return rc;
    if ((rc = dev_alloc(&L.blk_p0, p0.size()))) return rc;
    if (!p0.empty() && (rc = upload(L.blk_p0, p0.data(), sizeof(int32_t) * p0.size()))) return rc;
    if ((rc = dev_alloc(&L.win, wins.size()))) return rc;
    if (!wins.empty() && (rc = upload(L.win, wins.data(), sizeof(int4) * wins.size()))) return rc;
    if ((rc = dev_alloc(&L.blk_win, blk_win.size()))) return rc;
    if ((rc = upload(L.blk_win, blk_win.data(), sizeof(int32_t) * blk_win.size()))) return rc;
    for (int v = 0; v < 2; ++v) {
        if ((rc = dev_alloc(&L.blk_count[v], iblocks.size()))) return rc;
        if (hipMemset(L.blk_count[v], 0, sizeof(int32_t) * std::max<size_t>(iblocks.size(), 1)) != hipSuccess)
            return fail(GBR_E_HIP, "clearing the packing counts");
        if ((rc = dev_alloc(&L.run[v], (size_t)(L.n_intra + cap)))) return rc;
        if (!intra.empty() && (rc = upload(L.run[v], intra.data(), sizeof(int2) * intra.size()))) return rc;
        if ((rc = dev_alloc(&L.pk_hdr[v], std::max<size_t>((size_t)cap, 1)))) return rc;
        if ((rc = dev_alloc(&L.pk_j[v], std::max<size_t>((size_t)cap * 64, 1)))) return rc;
        L.n_run[v] = c->pack_count + 2 * k + v;
    }
    return GBR_OK;
}

}  // namespace

extern "C" {

const char* gbr_last_error(void) { return g_last_error.c_str(); }

int gbr_ctx_create(gbr_ctx** out, const gbr_gb_params* params, int32_t n_rep,
                   const int32_t* atom_off_host) {
    if (!out) return fail(GBR_E_INVAL, "out is null");
    *out = nullptr;
    if (!params) return fail(GBR_E_INVAL, "params is null");
    if (n_rep < 1 || n_rep >= gbr::MAX_REPLICAS) return fail(GBR_E_INVAL, "n_rep out of range");
    if (!atom_off_host) return fail(GBR_E_INVAL, "atom_off_host is null");
    if (atom_off_host[0] != 0) return fail(GBR_E_INVAL, "atom_off[0] must be 0");
    int64_t pairs = 0;
    int32_t max_n = 0;
    for (int r = 0; r < n_rep; ++r) {
        // in 64 bits: the difference of two arbitrary int32 offsets can overflow int32
        const int64_t n = (int64_t)atom_off_host[r + 1] - atom_off_host[r];
        if (n < 1) return fail(GBR_E_INVAL, "replica %d has %lld atoms", r, (long long)n);
        if (n > 64 * gbr::MAX_TILES) return fail(GBR_E_INVAL, "replica %d too large", r);
        max_n = std::max(max_n, (int32_t)n);
        pairs += (int64_t)n * (n - 1) / 2;
    }
    if (atom_off_host[n_rep] > GBR_MAX_ATOMS)
        return fail(GBR_E_INVAL, "%d atoms in the batch; at most %d", atom_off_host[n_rep], GBR_MAX_ATOMS);
    const gbr_gb_params& p = *params;
    if (!(p.k_e > 0) || !(p.eps_in > 0) || !(p.eps_out > 0) || !(p.offset >= 0))
        return fail(GBR_E_INVAL, "GB parameters out of range");
    if (!(p.kappa >= 0 && p.kappa <= 100) || !(p.cut >= 0 && p.cut <= 1e6) ||
        !(p.rgbmax >= 0 && p.rgbmax <= 1e6))
        return fail(GBR_E_INVAL, "kappa, cut and rgbmax must be finite and >= 0");
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1)
        return fail(GBR_E_NODEVICE, "no HIP device");
    int dev = 0;
    GBR_HIP(hipGetDevice(&dev));
    hipDeviceProp_t prop;
    GBR_HIP(hipGetDeviceProperties(&prop, dev));
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(GBR_E_NODEVICE, "device %d is %s; this library is built for gfx950", dev,
                    prop.gcnArchName);

    {
        NoallocDev nd;   // set-up of gb_born_radii_noalloc's scratch on this device
        if (int rc = noalloc_device(dev, &nd)) return rc;
    }
    gbr_ctx* c = new gbr_ctx();
    c->device = dev;
    c->n_cu = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
    c->prm = p;
    c->n_rep = n_rep;
    c->n_atoms = atom_off_host[n_rep];
    c->max_n = max_n;
    c->n_pairs = pairs;
    c->h_atom_off.assign(atom_off_host, atom_off_host + n_rep + 1);
    const int N = c->n_atoms;
    int rc = GBR_OK;
    auto done = [&](int code) { if (code) { gbr_ctx_destroy(c); } return code; };
    if ((rc = dev_alloc(&c->atom_off, n_rep + 1))) return done(rc);
    if ((rc = upload(c->atom_off, atom_off_host, sizeof(int32_t) * (n_rep + 1)))) return done(rc);
    std::vector<int2> tl;
    for (int r = 0; r < n_rep; ++r) {
        const int n = atom_off_host[r + 1] - atom_off_host[r];
        for (int t = 0; t < (n + 63) / 64; ++t) tl.push_back(make_int2(r, t));
    }
    c->n_tiles = (int32_t)tl.size();
    if ((rc = dev_alloc(&c->tiles, tl.size()))) return done(rc);
    if ((rc = upload(c->tiles, tl.data(), sizeof(int2) * tl.size()))) return done(rc);
    // with both cutoffs the pair passes run packed lists
    c->packed = p.cut > 0 && p.rgbmax > 0;
    if (c->packed) {
        std::vector<int32_t> tb(n_rep);
        for (int r = 0, t = 0; r < n_rep; ++r) {
            tb[r] = t;
            t += (atom_off_host[r + 1] - atom_off_host[r] + 63) / 64;
        }
        if ((rc = dev_alloc(&c->tile_base, n_rep))) return done(rc);
        if ((rc = upload(c->tile_base, tb.data(), sizeof(int32_t) * n_rep))) return done(rc);
        if ((rc = dev_alloc(&c->tile_box, 2 * (size_t)c->n_tiles))) return done(rc);
        if ((rc = dev_alloc(&c->pack_count, 8))) return done(rc);
    }
    for (int k = 0; k < 4; ++k)
        if ((rc = build_list(c, k))) return done(rc);
    // default register blocking: more i atoms per lane for larger replicas
    const int ni = max_n >= 4096 ? 8 : (max_n >= 512 ? 4 : (max_n >= 128 ? 2 : 1));
    c->ni_born = c->ni_energy = c->ni_chain = ni;
    if ((rc = dev_alloc(&c->psi_fx, N))) return done(rc);
    if ((rc = dev_alloc(&c->dEdR_fx, N))) return done(rc);
    if ((rc = dev_alloc(&c->dEdR, N))) return done(rc);
    if ((rc = dev_alloc(&c->chain_c, N))) return done(rc);
    if ((rc = dev_alloc(&c->ke_fx, n_rep))) return done(rc);
    if ((rc = dev_alloc(&c->ex_nH, n_rep))) return done(rc);
    if ((rc = dev_alloc(&c->ex_ne, n_rep))) return done(rc);
    if ((rc = dev_alloc(&c->ex_eps, n_rep))) return done(rc);
    if ((rc = dev_alloc(&c->ex_vscale, n_rep))) return done(rc);
    if ((rc = dev_alloc(&c->ex_enb, n_rep))) return done(rc);
    if ((rc = dev_alloc(&c->ex_fscale, n_rep))) return done(rc);
    if ((rc = dev_alloc(&c->mc_acc_fx, n_rep))) return done(rc);
    const size_t n_stripe = (size_t)n_rep * E_STRIPES * E_STRIPE_LEN;
    if ((rc = dev_alloc(&c->e_stripe, n_stripe))) return done(rc);
    if ((rc = dev_alloc(&c->step, 2))) return done(rc);
    if ((rc = dev_alloc(&c->err, 1))) return done(rc);
    hipError_t e = hipMemset(c->err, 0, sizeof(uint32_t));
    if (e == hipSuccess) e = hipMemset(c->mc_acc_fx, 0, sizeof(int64_t) * n_rep);
    if (e == hipSuccess) e = hipMemset(c->e_stripe, 0, sizeof(int64_t) * n_stripe);
    if (e == hipSuccess) e = hipMemset(c->step, 0, 2 * sizeof(uint64_t));
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) return done(hip_fail(e, "context init"));
    *out = c;
    return GBR_OK;
}

int gbr_ctx_destroy(gbr_ctx* c) {
    if (!c) return GBR_OK;
    // wait for and free on the context's own device, whatever the caller has current
    int prev = -1;
    const bool have_prev = hipGetDevice(&prev) == hipSuccess;
    if (!have_prev || prev != c->device) (void)hipSetDevice(c->device);
    (void)hipDeviceSynchronize();
    const int c_dev = c->device;
    for (auto& g : c->graph) if (g) (void)hipGraphExecDestroy(g);
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    for (auto& ev : c->timer.pool) if (ev) (void)hipEventDestroy(ev);
    (void)hipFree(c->atom_off);
    (void)hipFree(c->tiles);
    for (auto& L : c->lists) free_list(L);
    (void)hipFree(c->tile_base);
    (void)hipFree(c->tile_box);
    (void)hipFree(c->pack_count);
    (void)hipFree(c->psi_fx); (void)hipFree(c->dEdR_fx); (void)hipFree(c->dEdR); (void)hipFree(c->chain_c);
    (void)hipFree(c->ke_fx); (void)hipFree(c->ex_nH); (void)hipFree(c->ex_ne); (void)hipFree(c->ex_eps);
    (void)hipFree(c->ex_vscale); (void)hipFree(c->ex_enb); (void)hipFree(c->ex_fscale);
    (void)hipFree(c->mc_acc_fx); (void)hipFree(c->e_stripe);
    (void)hipFree(c->step); (void)hipFree(c->err);
    delete c;
    if (have_prev && prev != c_dev) (void)hipSetDevice(prev);
    return GBR_OK;
}

int gbr_ctx_sizes(const gbr_ctx* c, int32_t* n_atoms, int32_t* n_rep, int64_t* n_pairs) {
    if (int rc = check_ctx(c)) return rc;
    if (n_atoms) *n_atoms = c->n_atoms;
    if (n_rep) *n_rep = c->n_rep;
    if (n_pairs) *n_pairs = c->n_pairs;
    return GBR_OK;
}

int gbr_set_launch(gbr_ctx* c, int32_t waves_per_group, int32_t groups_per_cu) {
    if (int rc = check_ctx(c)) return rc;
    if (waves_per_group != 1 && waves_per_group != 2 && waves_per_group != 4)
        return fail(GBR_E_INVAL, "waves_per_group must be 1, 2 or 4");
    if (groups_per_cu < 1 || groups_per_cu > 32) return fail(GBR_E_INVAL, "groups_per_cu 1..32");
    c->shape.waves_per_group = waves_per_group;
    c->shape.groups_per_cu = groups_per_cu;
    // captured step graphs hold the old grids
    for (auto& g : c->graph) if (g) { (void)hipGraphExecDestroy(g); g = nullptr; }
    return GBR_OK;
}

int gbr_set_blocking(gbr_ctx* c, int32_t ni_born, int32_t ni_energy, int32_t ni_chain) {
    if (int rc = check_ctx(c)) return rc;
    auto ok = [](int v) { return v == 1 || v == 2 || v == 4 || v == 8; };
    if (!ok(ni_born) || !ok(ni_energy) || !ok(ni_chain))
        return fail(GBR_E_INVAL, "i atoms per lane must be 1, 2, 4 or 8");
    c->ni_born = ni_born; c->ni_energy = ni_energy; c->ni_chain = ni_chain;
    for (auto& g : c->graph) if (g) { (void)hipGraphExecDestroy(g); g = nullptr; }
    return GBR_OK;
}

int gbr_set_split(gbr_ctx* c, int32_t split_den) {
    if (int rc = check_ctx(c)) return rc;
    if (split_den < 1 || split_den > 1024) return fail(GBR_E_INVAL, "split_den must be 1..1024");
    if (split_den == c->split_den) return GBR_OK;
    if (hipDeviceSynchronize() != hipSuccess) return fail(GBR_E_HIP, "synchronizing before the list rebuild");
    c->split_den = split_den;
    for (int k = 0; k < 4; ++k)
        if (int rc = build_list(c, k)) return rc;
    for (auto& g : c->graph) if (g) { (void)hipGraphExecDestroy(g); g = nullptr; }
    return GBR_OK;
}

int gbr_set_timing(gbr_ctx* c, int32_t kinds_mask) {
    if (int rc = check_ctx(c)) return rc;
    if (kinds_mask < 0 || kinds_mask >= (1 << GBR_K_COUNT))
        return fail(GBR_E_INVAL, "kinds_mask must be a subset of the GBR_K_* bits");
    c->timer.mask = kinds_mask;
    return GBR_OK;
}

int gbr_get_timing(gbr_ctx* c, double* ms_out, int64_t* count_out) {
    if (int rc = check_ctx(c)) return rc;
    Timer& t = c->timer;
    for (size_t i = 0; i + 1 < t.used; i += 2) {
        GBR_HIP(hipEventSynchronize(t.pool[i + 1]));
        float ms = 0.0f;
        GBR_HIP(hipEventElapsedTime(&ms, t.pool[i], t.pool[i + 1]));
        const int k = t.kind[i / 2];
        t.ms[k] += ms;
        t.count[k] += 1;
    }
    for (int k = 0; k < GBR_K_COUNT; ++k) {
        if (ms_out) ms_out[k] = t.ms[k];
        if (count_out) count_out[k] = t.count[k];
        t.ms[k] = 0.0;
        t.count[k] = 0;
    }
    t.used = 0;
    t.kind.clear();
    return GBR_OK;
}

int gbr_check(gbr_ctx* c, hipStream_t stream, uint32_t* bits_out) {
    if (int rc = check_ctx(c)) return rc;
    GBR_HIP(hipStreamSynchronize(stream));
    uint32_t bits = 0;
    GBR_HIP(hipMemcpy(&bits, c->err, sizeof(bits), hipMemcpyDeviceToHost));
    GBR_HIP(hipMemset(c->err, 0, sizeof(uint32_t)));
    GBR_HIP(hipDeviceSynchronize());
    if (bits_out) *bits_out = bits;
    if (bits) return fail(GBR_E_NUMERIC, "device error word 0x%x", bits);
    return GBR_OK;
}

int gb_born_radii(gbr_ctx* c, const float* xyz, const float* rho, const float* screen, float* R,
                  float* dRdpsi, double* psi, hipStream_t s) {
    if (int rc = check_ctx(c)) return rc;
    REQ(xyz); REQ(rho); REQ(screen); REQ(R); REQ(dRdpsi);
    hipError_t e = launch_pack(c, xyz, s);
    if (e == hipSuccess) e = launch_zero_i64(c->psi_fx, c->n_atoms, s);
    if (e != hipSuccess) return hip_fail(e, "zero");
    {
        Timed t(c, GBR_K_BORN_PAIR, s, true);
        e = launch_born_pair(c, xyz, rho, screen, s, t.ev);
    }
    if (e != hipSuccess) return hip_fail(e, "born pair");
    {
        Timed t(c, GBR_K_PER_ATOM, s);
        e = launch_born_finalize(c, rho, R, dRdpsi, psi, s);
    }
    if (e != hipSuccess) return hip_fail(e, "born finalize");
    return GBR_OK;
}

int gb_born_radii_noalloc(const gbr_gb_params* params, int32_t n_rep, const int32_t* atom_off,
                          int32_t n_atoms, int32_t max_atoms, const float* xyz, const float* rho,
                          const float* screen, float* R, float* dRdpsi, double* psi, uint32_t* err,
                          hipStream_t s) {
    REQ(params); REQ(atom_off); REQ(xyz); REQ(rho); REQ(screen); REQ(R); REQ(dRdpsi); REQ(err);
    if (n_rep < 1 || n_rep >= gbr::MAX_REPLICAS) return fail(GBR_E_INVAL, "n_rep out of range");
    if (n_atoms < 1 || n_atoms > GBR_NOALLOC_MAX_ATOMS)
        return fail(GBR_E_INVAL, "n_atoms = %d: gb_born_radii_noalloc takes 1 .. %d atoms (its static scratch)",
                    n_atoms, GBR_NOALLOC_MAX_ATOMS);
    if (max_atoms < 1 || max_atoms > n_atoms)
        return fail(GBR_E_INVAL, "max_atoms = %d must lie in 1 .. n_atoms", max_atoms);
    const int T = (max_atoms + 63) / 64;
    if ((int64_t)n_rep * T * T >= (int64_t)1 << 31)
        return fail(GBR_E_INVAL, "n_rep x (max_atoms / 64)^2 too large for one launch");
    const gbr_gb_params& p = *params;
    if (!(p.offset >= 0) || !(p.alpha == p.alpha && p.beta == p.beta && p.gamma == p.gamma) ||
        !(p.rgbmax >= 0 && p.rgbmax <= 1e6))
        return fail(GBR_E_INVAL, "GB parameters out of range");
    int dev = 0;
    GBR_HIP(hipGetDevice(&dev));
    NoallocDev nd;
    if (int rc = noalloc_device(dev, &nd)) return rc;
    hipError_t e = launch_zero_i64(nd.scratch, n_atoms, s);
    if (e == hipSuccess)
        e = launch_born_pair_gen(p, n_rep, T, atom_off, n_atoms, nd.n_cu, xyz, rho, screen, nd.scratch, err, s);
    if (e == hipSuccess)
        e = launch_born_finalize_flat(p, n_atoms, n_rep, atom_off, rho, nd.scratch, R, dRdpsi, psi, err, s);
    if (e != hipSuccess) return hip_fail(e, "gb_born_radii_noalloc");
    return GBR_OK;
}

int gb_energy_forces(gbr_ctx* c, const float* xyz, const float* q, const float* rho,
                     const float* screen, const float* sigma, const float* eps, const float* R,
                     const float* dRdpsi, const double* psi, int64_t* force_fx,
                     int64_t* energy_fx, int32_t flags, int64_t* dEdq_fx, int64_t* dEdrho_fx,
                     hipStream_t s) {
    if (int rc = check_ctx(c)) return rc;
    REQ(xyz); REQ(q); REQ(rho); REQ(screen); REQ(sigma); REQ(eps); REQ(R); REQ(dRdpsi);
    REQ(force_fx); REQ(energy_fx);
    if (flags & ~(GBR_GRAD_Q | GBR_GRAD_RHO | GBR_ZERO_OUT))
        return fail(GBR_E_INVAL, "unknown flag bits 0x%x", flags);
    const bool gq = flags & GBR_GRAD_Q, gr = flags & GBR_GRAD_RHO;
    if (gq) REQ(dEdq_fx);
    if (gr) { REQ(dEdrho_fx); REQ(psi); }
    const int N = c->n_atoms;
    hipError_t e = hipSuccess;
    if (flags & GBR_ZERO_OUT) {
        e = launch_zero_i64(force_fx, 3ll * N, s);
        if (e == hipSuccess) e = launch_zero_i64(energy_fx, 4ll * c->n_rep, s);
        if (e == hipSuccess && gq) e = launch_zero_i64(dEdq_fx, N, s);
        if (e == hipSuccess && gr) e = launch_zero_i64(dEdrho_fx, N, s);
    }
    if (e == hipSuccess) e = launch_zero_i64(c->dEdR_fx, N, s);
    if (e == hipSuccess) e = launch_pack(c, xyz, s);
    if (e != hipSuccess) return hip_fail(e, "zero");
    {
        Timed t(c, GBR_K_ENERGY_PAIR, s, true);
        e = launch_energy_pair(c, xyz, q, R, sigma, eps, force_fx, gq ? dEdq_fx : nullptr, s, t.ev);
    }
    if (e != hipSuccess) return hip_fail(e, "energy pair");
    {
        Timed t(c, GBR_K_PER_ATOM, s);
        e = launch_coef(c, q, rho, R, dRdpsi, energy_fx, gq ? dEdq_fx : nullptr, nullptr, s);
    }
    if (e != hipSuccess) return hip_fail(e, "coef");
    {
        Timed t(c, GBR_K_CHAIN_PAIR, s, true);
        e = launch_chain_pair(c, xyz, rho, screen, force_fx, gr ? dEdrho_fx : nullptr, s, t.ev);
    }
    if (e != hipSuccess) return hip_fail(e, "chain pair");
    if (gr) {
        Timed t(c, GBR_K_PER_ATOM, s);
        e = launch_rho_finalize(c, rho, R, dRdpsi, psi, dEdrho_fx, s);
        if (e != hipSuccess) return hip_fail(e, "rho finalize");
    }
    return GBR_OK;
}

int titration_delta_e(gbr_ctx* c, const float* xyz, const float* q, const float* R,
                      const gbr_sites* sites, const int32_t* cand, int32_t n_cand, double* dE,
                      hipStream_t s) {
    if (int rc = check_ctx(c)) return rc;
    REQ(xyz); REQ(q); REQ(R); REQ(sites);
    if (n_cand < 0) return fail(GBR_E_INVAL, "n_cand < 0");
    if (n_cand == 0) return GBR_OK;
    REQ(cand); REQ(dE);
    if (int rc = check_sites(c, *sites)) return rc;
    if (sites->n_sites == 0) return fail(GBR_E_INVAL, "no sites");
    hipError_t e;
    {
        Timed t(c, GBR_K_TITRATION, s);
        e = launch_titration(c, xyz, q, R, *sites, cand, n_cand, dE, s);
    }
    if (e != hipSuccess) return hip_fail(e, "titration");
    return GBR_OK;
}

int remd_exchange(gbr_ctx* c, const gbr_grid* grid, uint64_t attempt, const int32_t* nH,
                  const int32_t* ne, const double* epsT, const double* enb, int32_t* target_idx,
                  int32_t* grid_rep, float* vscale, uint32_t* ex_stats, uint64_t seed,
                  hipStream_t s) {
    if (int rc = check_ctx(c)) return rc;
    REQ(grid); REQ(nH); REQ(ne); REQ(epsT); REQ(target_idx); REQ(grid_rep); REQ(vscale);
    if (int rc = check_grid(c, *grid)) return rc;
    if (grid->nHam > 1) REQ(enb);
    hipError_t e;
    {
        Timed t(c, GBR_K_EXCHANGE, s);
        e = launch_exchange(c, *grid, attempt, nullptr, 1, nH, ne, epsT, enb, target_idx, grid_rep,
                            vscale, nullptr, ex_stats, seed, s);
    }
    if (e != hipSuccess) return hip_fail(e, "exchange");
    return GBR_OK;
}

int gbr_exchange_inputs(gbr_ctx* c, const gbr_md_state* st, const gbr_md_params* pr, int32_t* nH,
                        int32_t* ne, double* epsT, double* enb, hipStream_t s) {
    if (int rc = check_ctx(c)) return rc;
    REQ(st); REQ(pr); REQ(nH); REQ(ne); REQ(epsT);
    REQ(st->site_state); REQ(st->target_idx); REQ(st->energy_fx);
    if (int rc = check_sites(c, pr->sites)) return rc;
    if (int rc = check_grid(c, pr->grid)) return rc;
    hipError_t e = launch_exchange_inputs(c, *st, *pr, nH, ne, epsT, enb, s);
    if (e != hipSuccess) return hip_fail(e, "exchange inputs");
    return GBR_OK;
}

int gbr_fx_to_float(gbr_ctx* c, const int64_t* src, int32_t components, int32_t bits,
                    const double* scale, int32_t sign, float* dst, hipStream_t s) {
    if (int rc = check_ctx(c)) return rc;
    REQ(src); REQ(dst);
    if (components < 1 || components > 3) return fail(GBR_E_INVAL, "components must be 1..3");
    if (bits < 0 || bits > 62) return fail(GBR_E_INVAL, "bits must be 0..62");
    if (sign != 1 && sign != -1) return fail(GBR_E_INVAL, "sign must be +1 or -1");
    hipError_t e = launch_fx_to_float(c, src, components, bits, scale, sign, dst, s);
    if (e != hipSuccess) return hip_fail(e, "fx to float");
    return GBR_OK;
}

int gbr_energies(gbr_ctx* c, const int64_t* energy_fx, double* out, hipStream_t s) {
    if (int rc = check_ctx(c)) return rc;
    REQ(energy_fx); REQ(out);
    hipError_t e = launch_energies(c, energy_fx, out, s);
    if (e != hipSuccess) return hip_fail(e, "energies");
    return GBR_OK;
}

int md_step(gbr_ctx* c, gbr_md_state* st, const gbr_md_params* pr, uint64_t seed, uint64_t step0,
            int32_t n_steps, int32_t flags, hipStream_t s) {
    if (int rc = check_ctx(c)) return rc;
    REQ(st); REQ(pr);
    REQ(st->xyz); REQ(st->v); REQ(st->q); REQ(st->force_fx); REQ(st->energy_fx); REQ(st->R);
    REQ(st->dRdpsi); REQ(st->target_idx); REQ(st->grid_rep);
    REQ(pr->rho); REQ(pr->screen); REQ(pr->sigma); REQ(pr->eps); REQ(pr->mass); REQ(pr->x0);
    if (n_steps < 0) return fail(GBR_E_INVAL, "n_steps < 0");
    if (flags & ~(GBR_MD_INIT_FORCES | GBR_MD_GRAPH)) return fail(GBR_E_INVAL, "unknown md flags");
    if (!(pr->dt >= 0) || !(pr->gamma >= 0)) return fail(GBR_E_INVAL, "dt and gamma must be >= 0");
    if (pr->mc_every < 0 || pr->ex_every < 0) return fail(GBR_E_INVAL, "intervals must be >= 0");
    if (int rc = check_grid(c, pr->grid)) return rc;
    if (int rc = check_sites(c, pr->sites)) return rc;
    if (pr->mc_every > 0 && pr->sites.n_sites > 0) REQ(st->site_state);
    if (pr->ex_every > 0 && pr->sites.n_sites > 0) REQ(st->site_state);
    if (pr->sites.n_sites == 0 && pr->mc_every > 0)
        return fail(GBR_E_INVAL, "mc_every > 0 needs titratable sites");
    MDArgs a{*st, *pr, seed};
    hipError_t e = launch_set_step(c, step0, s);
    if (e != hipSuccess) return hip_fail(e, "set step");
    if (flags & GBR_MD_INIT_FORCES) {
        e = launch_zero_i64(st->force_fx, 3ll * c->n_atoms, s);
        if (e == hipSuccess) e = launch_zero_i64(st->energy_fx, 4ll * c->n_rep, s);
        if (e == hipSuccess) e = launch_zero_i64(c->psi_fx, c->n_atoms, s);
        if (e == hipSuccess) e = launch_zero_i64(c->dEdR_fx, c->n_atoms, s);
        if (e == hipSuccess) e = launch_zero_i64(c->ke_fx, c->n_rep, s);
        if (e != hipSuccess) return hip_fail(e, "zero");
        if (int rc = md_forces(c, a, false, false, s)) return rc;
        e = launch_md_last(c, a, 0, s);
        if (e != hipSuccess) return hip_fail(e, "md init");
    }
    const bool use_graph = (flags & GBR_MD_GRAPH) != 0 && c->timer.mask == 0;
    uint64_t key = use_graph ? hash_args(a) : 0;
    bool prev_open = false;            // the previous step still needs its closing half
    for (int32_t k = 0; k < n_steps; ++k) {
        const uint64_t n = step0 + (uint64_t)k;
        int kind = 0;
        if (pr->mc_every > 0 && (n + 1) % (uint64_t)pr->mc_every == 0) kind |= STEP_MC;
        if (pr->ex_every > 0 && (n + 1) % (uint64_t)pr->ex_every == 0) kind |= STEP_EX | STEP_LAST;
        if (k == n_steps - 1) kind |= STEP_LAST;
        if (prev_open) kind |= STEP_MID;
        prev_open = !(kind & STEP_LAST);
        if (!use_graph) {
            if (int rc = md_one_step(c, a, kind, s)) return rc;
            continue;
        }
        if (!c->graph[kind] || c->graph_key[kind] != key) {
            if (c->graph[kind]) { (void)hipGraphExecDestroy(c->graph[kind]); c->graph[kind] = nullptr; }
            if (!c->cap_stream) GBR_HIP(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
            GBR_HIP(hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
            int rc = md_one_step(c, a, kind, c->cap_stream);
            hipGraph_t g = nullptr;
            hipError_t ec = hipStreamEndCapture(c->cap_stream, &g);
            if (rc) { if (g) (void)hipGraphDestroy(g); return rc; }
            if (ec != hipSuccess) return hip_fail(ec, "end capture");
            hipError_t ei = hipGraphInstantiate(&c->graph[kind], g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            if (ei != hipSuccess) return hip_fail(ei, "graph instantiate");
            c->graph_key[kind] = key;
        }
        GBR_HIP(hipGraphLaunch(c->graph[kind], s));
    }
    e = launch_ke_out(c, st->ke, s);
    if (e != hipSuccess) return hip_fail(e, "kinetic energy");
    return GBR_OK;
}

}  // extern "C"
