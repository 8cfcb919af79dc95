"""Python layer over the C ABI: a context bound to one batch layout, device
copies of a batch, the autograd Function, and the md_step wrapper (MD).

Torch provides device memory and streams; every computation is a call into
libgbremd.so (HIP kernels).  Results come back as torch tensors.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass, field

import numpy as np
import torch

from . import _capi as A
from ._capi import check, ptr, stream_handle

F32, F64, I32, I64 = torch.float32, torch.float64, torch.int32, torch.int64


class Context:
    """A gbr_ctx for one batch layout (replicas back to back, atom_off on the host)."""

    def __init__(self, atom_off, params: A.GBParams | None = None, device=None):
        self.device = torch.device(device or "cuda")
        off = np.ascontiguousarray(np.asarray(atom_off, dtype=np.int32))
        self.atom_off = off
        self.n_rep = off.size - 1
        self.n_atoms = int(off[-1])
        self.params = params or A.obc2()
        h = C.c_void_p()
        with torch.cuda.device(self.device):
            check(A.lib.gbr_ctx_create(C.byref(h), C.byref(self.params), self.n_rep,
                                       off.ctypes.data_as(C.POINTER(C.c_int32))))
        self.h = h
        npairs = C.c_int64()
        check(A.lib.gbr_ctx_sizes(self.h, None, None, C.byref(npairs)))
        self.n_pairs = int(npairs.value)

    def close(self):
        if getattr(self, "h", None):
            A.lib.gbr_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---------------------------------------------------------------- config
    def set_launch(self, waves_per_group=4, groups_per_cu=8):
        check(A.lib.gbr_set_launch(self.h, waves_per_group, groups_per_cu))

    def set_blocking(self, ni_born, ni_energy, ni_chain):
        check(A.lib.gbr_set_blocking(self.h, ni_born, ni_energy, ni_chain))

    def set_split(self, split_den=16):
        check(A.lib.gbr_set_split(self.h, split_den))

    def set_timing(self, on, kinds=None):
        """Time kernels with HIP events: all kinds when on is True, or only the
        named kinds (see _capi.KERNEL_KINDS)."""
        mask = 0
        if on:
            names = kinds or A.KERNEL_KINDS
            for k in names:
                mask |= 1 << A.KERNEL_KINDS.index(k)
        check(A.lib.gbr_set_timing(self.h, mask))

    def get_timing(self):
        ms = (C.c_double * A.K_COUNT)()
        cnt = (C.c_int64 * A.K_COUNT)()
        check(A.lib.gbr_get_timing(self.h, ms, cnt))
        return {k: (ms[i], cnt[i]) for i, k in enumerate(A.KERNEL_KINDS)}

    def check(self, stream=None):
        """Synchronize and raise if the device error word is set."""
        bits = C.c_uint32()
        rc = A.lib.gbr_check(self.h, stream_handle(stream), C.byref(bits))
        if rc == A.GBR_E_NUMERIC:
            raise A.GBRError(rc, f"device error bits 0x{bits.value:x}")
        check(rc)

    # ------------------------------------------------------------ the path
    def _new(self, shape, dtype):
        return torch.empty(shape, dtype=dtype, device=self.device)

    def born_radii(self, xyz, rho, screen, want_psi=True, out=None, stream=None):
        N = self.n_atoms
        R, dR = (out or (self._new(N, F32), self._new(N, F32)))
        psi = self._new(N, F64) if want_psi else None
        check(A.lib.gb_born_radii(self.h, ptr(xyz, F32, 3 * N, "xyz"), ptr(rho, F32, N, "rho"),
                                  ptr(screen, F32, N, "screen"), ptr(R, F32, N), ptr(dR, F32, N),
                                  ptr(psi, F64, N), stream_handle(stream)))
        return R, dR, psi

    def energy_forces(self, xyz, q, rho, screen, sigma, eps, R, dRdpsi, psi=None,
                      grad_q=False, grad_rho=False, stream=None):
        """Returns (force_fx [3N] int64, energy_fx [4 n_rep] int64, dEdq_fx, dEdrho_fx)."""
        N = self.n_atoms
        f = torch.zeros(3 * N, dtype=I64, device=self.device)
        e = torch.zeros(4 * self.n_rep, dtype=I64, device=self.device)
        dq = torch.zeros(N, dtype=I64, device=self.device) if grad_q else None
        dr = torch.zeros(N, dtype=I64, device=self.device) if grad_rho else None
        flags = (A.GRAD_Q if grad_q else 0) | (A.GRAD_RHO if grad_rho else 0)
        check(A.lib.gb_energy_forces(
            self.h, ptr(xyz, F32, 3 * N, "xyz"), ptr(q, F32, N, "q"), ptr(rho, F32, N, "rho"),
            ptr(screen, F32, N, "screen"), ptr(sigma, F32, N, "sigma"), ptr(eps, F32, N, "eps"),
            ptr(R, F32, N, "R"), ptr(dRdpsi, F32, N, "dRdpsi"), ptr(psi, F64, N, "psi"),
            ptr(f), ptr(e), flags, ptr(dq), ptr(dr), stream_handle(stream)))
        return f, e, dq, dr

    def energies(self, energy_fx, stream=None):
        """[n_rep, 5] doubles: E_GB, E_C, E_LJ, slot 3, E_GB + E_C + E_LJ."""
        out = self._new((self.n_rep, 5), F64)
        check(A.lib.gbr_energies(self.h, ptr(energy_fx, I64, 4 * self.n_rep), ptr(out),
                                 stream_handle(stream)))
        return out

    def fx_to_float(self, src, components, bits=A.FX_BITS_FORCE, scale=None, sign=1, stream=None):
        dst = self._new(src.numel(), F32)
        check(A.lib.gbr_fx_to_float(self.h, ptr(src, I64, components * self.n_atoms), components,
                                    bits, ptr(scale, F64, self.n_rep, "scale"), sign, ptr(dst),
                                    stream_handle(stream)))
        return dst

    def titration_delta_e(self, xyz, q, R, sites: "DeviceBatch", cand, stream=None):
        cand = cand.to(device=self.device, dtype=I32).contiguous()
        n = cand.numel() // 2
        dE = self._new(n, F64)
        check(A.lib.titration_delta_e(self.h, ptr(xyz, F32, 3 * self.n_atoms), ptr(q, F32),
                                      ptr(R, F32), C.byref(sites.sites), ptr(cand), n, ptr(dE),
                                      stream_handle(stream)))
        return dE

    def remd_exchange(self, grid: A.Grid, attempt, nH, ne, epsT, target_idx, grid_rep, seed,
                      ex_stats=None, enb=None, stream=None):
        vscale = self._new(self.n_rep, F32)
        check(A.lib.remd_exchange(self.h, C.byref(grid), int(attempt), ptr(nH, I32), ptr(ne, I32),
                                  ptr(epsT, F64), ptr(enb, F64), ptr(target_idx, I32), ptr(grid_rep, I32),
                                  ptr(vscale), ptr(ex_stats, torch.int32), int(seed),
                                  stream_handle(stream)))
        return vscale


# --------------------------------------------------------------------- batch
@dataclass
class DeviceBatch:
    """Device copies of a synthetic (or user) batch plus the C structures
    pointing into them.  Keys follow the generator's dict."""
    t: dict
    sites: A.Sites
    grid: A.Grid
    n_rep: int
    n_atoms: int
    keep: list = field(default_factory=list)

    @staticmethod
    def from_numpy(b: dict, device="cuda"):
        dev = torch.device(device)
        t = {}

        def put(key, arr, dtype):
            t[key] = torch.as_tensor(np.ascontiguousarray(arr)).to(device=dev, dtype=dtype).contiguous()

        soa = lambda a: np.asarray(a, dtype=np.float32).T.reshape(-1)   # [N,3] -> x..,y..,z..
        put("xyz", soa(b["xyz"]), F32)
        put("x0", soa(b["x0"]), F32)
        put("v", soa(b.get("v", np.zeros_like(b["xyz"]))), F32)
        for k in ("q", "rho", "screen", "sigma", "eps", "mass"):
            put(k, b[k], F32)
        ns = int(b["n_sites"])
        if ns > 0:
            for k in ("rep_site_off", "site_off", "site_atoms", "site_type", "n_states",
                      "state_nH", "state_ne", "site_state"):
                put(k, b[k], I32)
            put("site_rep", b.get("site_rep", np.repeat(np.arange(b["n_rep"]),
                                                          np.diff(b["rep_site_off"]))), I32)
            put("state_q", b["state_q"], F32)
            put("G_ref", b["G_ref"], F64)
            put("ref_value", b["ref_value"], F64)
        for k in ("E_vals", "pH_vals", "T_vals", "H_scale"):
            put(k, b.get(k, [1.0]) if k == "H_scale" else b[k], F64)
        put("target_idx", np.asarray(b["target_idx"]).reshape(-1), I32)
        put("grid_rep", b["grid_rep"], I32)
        sites = A.Sites()
        sites.n_sites = ns
        sites.max_states = int(b["max_states"])
        if ns > 0:
            for k in ("rep_site_off", "site_off", "site_atoms", "site_rep", "site_type",
                      "n_states", "state_q", "state_nH", "state_ne", "G_ref", "ref_value"):
                setattr(sites, k, t[k].data_ptr())
        grid = A.Grid()
        grid.n_inst = int(b["n_inst"])
        grid.nE, grid.npH, grid.nT = len(b["E_vals"]), len(b["pH_vals"]), len(b["T_vals"])
        grid.nHam = t["H_scale"].numel()
        grid.E_vals, grid.pH_vals, grid.T_vals = (t["E_vals"].data_ptr(), t["pH_vals"].data_ptr(),
                                                  t["T_vals"].data_ptr())
        grid.H_scale = t["H_scale"].data_ptr()
        order = list(b["dim_order"])
        grid.n_dims = len(order)
        for k in range(A.N_DIMS):
            grid.dim_order[k] = order[k] if k < len(order) else 0
        return DeviceBatch(t, sites, grid, int(b["n_rep"]), int(b["atom_off"][-1]))

    def set_G_ref(self, G_ref):
        self.t["G_ref"].copy_(torch.as_tensor(G_ref, dtype=F64))


class MD:
    """md_step on a DeviceBatch: owns the state tensors and the C structures."""

    def __init__(self, ctx: Context, batch: DeviceBatch, b: dict, seed: int, eps_mode=0,
                 stats=True):
        self.ctx, self.batch = ctx, batch
        N, R = ctx.n_atoms, ctx.n_rep
        dev = ctx.device
        t = batch.t
        self.force_fx = torch.zeros(3 * N, dtype=I64, device=dev)
        self.energy_fx = torch.zeros(4 * R, dtype=I64, device=dev)
        self.R = torch.zeros(N, dtype=F32, device=dev)
        self.dRdpsi = torch.zeros(N, dtype=F32, device=dev)
        self.ke = torch.zeros(R, dtype=F64, device=dev)
        ns = batch.sites.n_sites
        G = R                   # one grid point per replica
        self.mc_stats = torch.zeros(2 * max(ns, 1), dtype=torch.int32, device=dev) if stats else None
        self.ex_stats = torch.zeros(2 * A.N_DIMS * G, dtype=torch.int32, device=dev) if stats else None
        st = A.MDState()
        st.xyz, st.v, st.q = t["xyz"].data_ptr(), t["v"].data_ptr(), t["q"].data_ptr()
        st.force_fx, st.energy_fx = self.force_fx.data_ptr(), self.energy_fx.data_ptr()
        st.R, st.dRdpsi = self.R.data_ptr(), self.dRdpsi.data_ptr()
        st.site_state = t["site_state"].data_ptr() if ns > 0 else None
        st.target_idx, st.grid_rep = t["target_idx"].data_ptr(), t["grid_rep"].data_ptr()
        st.ke = self.ke.data_ptr()
        st.mc_stats = self.mc_stats.data_ptr() if stats else None
        st.ex_stats = self.ex_stats.data_ptr() if stats else None
        pr = A.MDParams()
        for k in ("rho", "screen", "sigma", "eps", "mass", "x0"):
            setattr(pr, k, t[k].data_ptr())
        pr.k_tether, pr.dt, pr.gamma = float(b["k_tether"]), float(b["dt"]), float(b["gamma_ps"])
        pr.mc_every, pr.ex_every, pr.eps_mode = int(b["mc_every"]), int(b["ex_every"]), int(eps_mode)
        pr.sites = batch.sites
        pr.grid = batch.grid
        self.st, self.pr, self.seed = st, pr, int(seed)
        self.step = 0

    def run(self, n_steps: int, init_forces=False, graph=False, stream=None):
        flags = (A.MD_INIT_FORCES if init_forces else 0) | (A.MD_GRAPH if graph else 0)
        check(A.lib.md_step(self.ctx.h, C.byref(self.st), C.byref(self.pr), self.seed, self.step,
                            int(n_steps), flags, stream_handle(stream)))
        self.step += int(n_steps)

    def exchange_inputs(self, stream=None):
        """(N_H, N_e, epsT, enb) per replica, as md_step's exchange reads them."""
        R = self.ctx.n_rep
        nH = torch.empty(R, dtype=I32, device=self.ctx.device)
        ne = torch.empty(R, dtype=I32, device=self.ctx.device)
        ep = torch.empty(R, dtype=F64, device=self.ctx.device)
        enb = torch.empty(R, dtype=F64, device=self.ctx.device)
        check(A.lib.gbr_exchange_inputs(self.ctx.h, C.byref(self.st), C.byref(self.pr), ptr(nH),
                                        ptr(ne), ptr(ep), ptr(enb), stream_handle(stream)))
        return nH, ne, ep, enb


# ------------------------------------------------------------- autograd
class GBEnergy(torch.autograd.Function):
    """E[r] = E_GB + E_C + E_LJ of every replica; gradients dE/dx (SoA 3N),
    dE/dq and dE/drho come from the library's adjoint (forces and the
    GRAD_Q / GRAD_RHO accumulators), scaled by the upstream gradient in the
    library's conversion kernel.  screen, sigma and eps are not
    differentiable.  Double backward is not supported."""

    @staticmethod
    def forward(fctx, xyz, q, rho, screen, sigma, eps, gctx: Context):
        for name, t in (("screen", screen), ("sigma", sigma), ("eps", eps)):
            if t.requires_grad:
                raise ValueError(f"GBEnergy is not differentiable with respect to {name}")
        xyz_, q_, rho_ = xyz.detach().contiguous(), q.detach().contiguous(), rho.detach().contiguous()
        R, dR, psi = gctx.born_radii(xyz_, rho_, screen)
        f, e, dq, dr = gctx.energy_forces(xyz_, q_, rho_, screen, sigma, eps, R, dR, psi,
                                          grad_q=True, grad_rho=True)
        E = gctx.energies(e)[:, 4].clone()
        fctx.gctx = gctx
        fctx.save_for_backward(f, dq, dr)
        fctx.mark_non_differentiable()
        return E

    @staticmethod
    def backward(fctx, gE):
        f, dq, dr = fctx.saved_tensors
        g = fctx.gctx
        scale = gE.detach().to(F64).contiguous()
        gx = g.fx_to_float(f, 3, scale=scale, sign=-1) if fctx.needs_input_grad[0] else None
        gq = g.fx_to_float(dq, 1, scale=scale) if fctx.needs_input_grad[1] else None
        gr = g.fx_to_float(dr, 1, scale=scale) if fctx.needs_input_grad[2] else None
        return gx, gq, gr, None, None, None, None


def gb_energy(xyz, q, rho, screen, sigma, eps, gctx: Context):
    return GBEnergy.apply(xyz, q, rho, screen, sigma, eps, gctx)


# --------------------------------------------------- reference energies
def reference_energies(b: dict, params: A.GBParams | None = None, device="cuda"):
    """G_ref per (site, state) for a batch: 0 for state 0 and, for the other
    states, the electrostatic energy change of the site's atoms alone (the
    reference compound, at the batch's starting geometry), evaluated with this
    library.  With these values an isolated site titrates at pKa_ref / E0_ref."""
    ms = int(b["max_states"])
    ns = int(b["n_sites"])
    out = np.zeros(ns * ms)
    if ns == 0:
        return out
    sizes = np.diff(b["site_off"])
    sub = {"atom_off": np.concatenate([[0], np.cumsum(sizes)]).astype(np.int32)}
    idx = np.asarray(b["site_atoms"])
    ctx = Context(sub["atom_off"], params, device)
    dev = ctx.device
    soa = lambda a: torch.as_tensor(np.asarray(a, np.float32).T.reshape(-1).copy(), device=dev)
    xyz = soa(b["xyz"][idx])
    rho = torch.as_tensor(b["rho"][idx], device=dev)
    scr = torch.as_tensor(b["screen"][idx], device=dev)
    q0 = torch.as_tensor(np.asarray(b["state_q"]).reshape(-1, ms)[:, 0].astype(np.float32), device=dev)
    R, _, _ = ctx.born_radii(xyz, rho, scr, want_psi=False)
    # candidates: (site, state) for every non-zero state, against state-0 charges
    cand = [(s, k) for s in range(ns) for k in range(1, int(b["n_states"][s]))]
    sd = {"n_sites": ns, "max_states": ms, "rep_site_off": np.arange(ns + 1, dtype=np.int32),
          "site_off": np.asarray(b["site_off"], np.int32),
          "site_atoms": np.arange(idx.size, dtype=np.int32),
          "site_rep": np.arange(ns, dtype=np.int32), "site_type": b["site_type"],
          "n_states": b["n_states"], "state_q": b["state_q"], "state_nH": b["state_nH"],
          "state_ne": b["state_ne"], "G_ref": np.zeros(ns * ms), "ref_value": b["ref_value"]}
    keep = {k: torch.as_tensor(np.ascontiguousarray(v), device=dev) for k, v in sd.items()
            if isinstance(v, np.ndarray)}
    keep["state_q"] = keep["state_q"].to(F32)
    keep["G_ref"] = keep["G_ref"].to(F64)
    keep["ref_value"] = keep["ref_value"].to(F64)
    for k in ("rep_site_off", "site_off", "site_atoms", "site_rep", "site_type", "n_states",
              "state_nH", "state_ne"):
        keep[k] = keep[k].to(I32)
    S = A.Sites()
    S.n_sites, S.max_states = ns, ms
    for k in ("rep_site_off", "site_off", "site_atoms", "site_rep", "site_type", "n_states",
              "state_q", "state_nH", "state_ne", "G_ref", "ref_value"):
        setattr(S, k, keep[k].data_ptr())
    holder = type("S", (), {})()
    holder.sites = S
    c = torch.as_tensor(np.asarray(cand, np.int32).reshape(-1), device=dev)
    dE = ctx.titration_delta_e(xyz, q0, R, holder, c)
    ctx.check()
    dE = dE.cpu().numpy()
    for (s, k), v in zip(cand, dE):
        out[s * ms + k] = v
    ctx.close()
    return out
