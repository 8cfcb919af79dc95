"""Plain double-precision CPU oracle (test infrastructure only).

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product library never does, and this
package imports nothing from the product: its arithmetic lives in
``gbr_oracle.c`` (plain C, FP64, O(N^2) loops in the order of the definitions)
and this module only marshals numpy arrays through ctypes.

Coordinates handed to the oracle are float64 arrays of shape [N, 3]; every
function promotes whatever it is given to float64 so that a float32 input is
used at exactly the value the GPU path sees.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gbr_oracle.c")
# GBR_ORACLE_LIB names another build of gbr_oracle.c to load (the sanitized
# build that the CPU sanitizer test makes); unset, the in-tree library
_LIB = os.environ.get("GBR_ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, no fast math, OpenMP over rows)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-Wall",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        _lib = C.CDLL(_LIB)
        _declare(_lib)
    return _lib


class GBParams(C.Structure):
    _fields_ = [("k_e", C.c_double), ("eps_in", C.c_double), ("eps_out", C.c_double),
                ("offset", C.c_double), ("alpha", C.c_double), ("beta", C.c_double),
                ("gamma", C.c_double), ("kappa", C.c_double), ("cut", C.c_double),
                ("rgbmax", C.c_double)]


def obc2(k_e=332.0522173, eps_in=1.0, eps_out=78.5, offset=0.09,
         alpha=1.0, beta=0.8, gamma=4.85, kappa=0.0, cut=0.0, rgbmax=0.0) -> GBParams:
    """OBC-II parameter set (igb=2); kappa (1/A) screens the GB term with salt,
    cut and rgbmax (A) truncate the pair energies and the descreening sum (0:
    no salt, no cutoff)."""
    return GBParams(k_e, eps_in, eps_out, offset, alpha, beta, gamma, kappa, cut, rgbmax)


_dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_ip = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_P = C.POINTER


class MDCfg(C.Structure):
    _fields_ = [
        ("n_rep", C.c_int), ("atom_off", _P(C.c_int)),
        ("n_sites", C.c_int), ("max_states", C.c_int),
        ("rep_site_off", _P(C.c_int)), ("site_off", _P(C.c_int)), ("site_atoms", _P(C.c_int)),
        ("site_type", _P(C.c_int)), ("n_states", _P(C.c_int)),
        ("state_q", _P(C.c_double)), ("state_nH", _P(C.c_int)), ("state_ne", _P(C.c_int)),
        ("G_ref", _P(C.c_double)), ("ref_value", _P(C.c_double)),
        ("n_inst", C.c_int), ("nE", C.c_int), ("npH", C.c_int), ("nT", C.c_int), ("nHam", C.c_int),
        ("E_vals", _P(C.c_double)), ("pH_vals", _P(C.c_double)), ("T_vals", _P(C.c_double)),
        ("H_scale", _P(C.c_double)),
        ("n_dims", C.c_int), ("dim_order", C.c_int * 4),
        ("rho", _P(C.c_double)), ("scr", _P(C.c_double)), ("sig", _P(C.c_double)),
        ("eps", _P(C.c_double)), ("mass", _P(C.c_double)), ("x0", _P(C.c_double)),
        ("gb", GBParams),
        ("k_tether", C.c_double), ("dt", C.c_double), ("gamma_ps", C.c_double),
        ("mc_every", C.c_int), ("ex_every", C.c_int), ("eps_mode", C.c_int),
        ("seed", C.c_uint64),
    ]


class MDState(C.Structure):
    _fields_ = [
        ("xyz", _P(C.c_double)), ("v", _P(C.c_double)), ("q", _P(C.c_double)),
        ("F", _P(C.c_double)), ("E", _P(C.c_double)),
        ("site_state", _P(C.c_int)), ("target_idx", _P(C.c_int)), ("grid_rep", _P(C.c_int)),
        ("mc_att", _P(C.c_longlong)), ("mc_acc", _P(C.c_longlong)),
        ("ex_att", _P(C.c_longlong)), ("ex_acc", _P(C.c_longlong)),
    ]


def _declare(L):
    L.orc_philox4x32_10.argtypes = [_P(C.c_uint32), _P(C.c_uint32), _P(C.c_uint32)]
    L.orc_uniform53.argtypes = [C.c_uint32, C.c_uint32]
    L.orc_uniform53.restype = C.c_double
    L.orc_normal2.argtypes = [_P(C.c_uint32), _P(C.c_double), _P(C.c_double)]
    L.orc_hct.argtypes = [C.c_double, C.c_double, C.c_double]
    L.orc_hct.restype = C.c_double
    L.orc_hct_grad.argtypes = [C.c_double, C.c_double, C.c_double,
                               _P(C.c_double), _P(C.c_double), _P(C.c_double)]
    L.orc_born.argtypes = [C.c_int, _dp, _dp, _dp, _P(GBParams), _dp, _dp, _dp]
    L.orc_energy.argtypes = [C.c_int, _dp, _dp, _dp, _dp, _dp, _P(GBParams), _dp]
    L.orc_elec_energy.argtypes = [C.c_int, _dp, _dp, _dp, _P(GBParams)]
    L.orc_elec_energy.restype = C.c_double
    for fn in (L.orc_delta_e_plain, L.orc_delta_e_incr, L.orc_delta_e_abs):
        fn.argtypes = [C.c_int, _dp, _dp, _dp, _P(GBParams), C.c_int, _ip, _dp]
        fn.restype = C.c_double
    L.orc_gradient.argtypes = [C.c_int, _dp, _dp, _dp, _dp, _dp, _dp, _P(GBParams),
                               _dp, _dp, _dp, _dp]
    L.orc_tether.argtypes = [C.c_int, _dp, _dp, C.c_double, _dp]
    L.orc_tether.restype = C.c_double
    L.orc_md_run.argtypes = [_P(MDCfg), _P(MDState), C.c_longlong, C.c_int, C.c_int]
    L.orc_md_run.restype = C.c_int
    L.orc_exchange.argtypes = [_P(MDCfg), C.c_longlong, _ip, _ip, _dp, _dp, _ip, _ip, _dp,
                               _P(C.c_longlong), _P(C.c_longlong)]
    L.orc_replica_counts.argtypes = [_P(MDCfg), _ip, _ip, _dp, C.c_int,
                                     _P(C.c_int), _P(C.c_int), _P(C.c_double)]
    L.orc_constants.argtypes = [_dp]


def _f64(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _i32(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.int32))


def constants() -> dict:
    out = np.zeros(4)
    lib().orc_constants(out)
    return {"kB": out[0], "F": out[1], "ln10": out[2], "conv": out[3]}


# ------------------------------------------------------------------ RNG
def philox(ctr, key):
    c = (C.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in ctr])
    k = (C.c_uint32 * 2)(*[int(v) & 0xFFFFFFFF for v in key])
    o = (C.c_uint32 * 4)()
    lib().orc_philox4x32_10(c, k, o)
    return [int(v) for v in o]


def uniform53(a, b) -> float:
    return lib().orc_uniform53(int(a) & 0xFFFFFFFF, int(b) & 0xFFFFFFFF)


def normal2(words):
    w = (C.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in words])
    a, b = C.c_double(), C.c_double()
    lib().orc_normal2(w, C.byref(a), C.byref(b))
    return a.value, b.value


# ------------------------------------------------------------------ GB
def hct(r, rt, s) -> float:
    return lib().orc_hct(float(r), float(rt), float(s))


def hct_grad(r, rt, s):
    a, b, c = C.c_double(), C.c_double(), C.c_double()
    lib().orc_hct_grad(float(r), float(rt), float(s), C.byref(a), C.byref(b), C.byref(c))
    return a.value, b.value, c.value


def born(xyz, rho, scr, gb=None):
    """Born radii of one system: returns (psi, R, dR/dpsi)."""
    gb = gb or obc2()
    xyz = _f64(xyz).reshape(-1)
    n = xyz.size // 3
    psi, R, d = np.zeros(n), np.zeros(n), np.zeros(n)
    lib().orc_born(n, xyz, _f64(rho), _f64(scr), C.byref(gb), psi, R, d)
    return psi, R, d


def energy_at_R(xyz, q, R, sig, eps, gb=None):
    """(E_GB, E_C, E_LJ) of one system at the given Born radii."""
    gb = gb or obc2()
    xyz = _f64(xyz).reshape(-1)
    E = np.zeros(3)
    lib().orc_energy(xyz.size // 3, xyz, _f64(q), _f64(R), _f64(sig), _f64(eps), C.byref(gb), E)
    return E


def elec_energy(xyz, q, R, gb=None) -> float:
    gb = gb or obc2()
    xyz = _f64(xyz).reshape(-1)
    return lib().orc_elec_energy(xyz.size // 3, xyz, _f64(q), _f64(R), C.byref(gb))


def delta_e(xyz, q, R, idx, qnew, gb=None, incremental=False) -> float:
    """Titration energy change when q[idx] becomes qnew, at fixed Born radii."""
    gb = gb or obc2()
    xyz = _f64(xyz).reshape(-1)
    idx = _i32(idx)
    fn = lib().orc_delta_e_incr if incremental else lib().orc_delta_e_plain
    return fn(xyz.size // 3, xyz, _f64(q), _f64(R), C.byref(gb), idx.size, idx, _f64(qnew))


def delta_e_abs_scale(xyz, q, R, idx, qnew, gb=None) -> float:
    """Sum of the absolute values of the incremental form's terms (an error
    scale for a titration energy change evaluated in lower precision)."""
    gb = gb or obc2()
    xyz = _f64(xyz).reshape(-1)
    idx = _i32(idx)
    return lib().orc_delta_e_abs(xyz.size // 3, xyz, _f64(q), _f64(R), C.byref(gb), idx.size, idx, _f64(qnew))


def gradient(xyz, q, rho, scr, sig, eps, gb=None):
    """Energy (E_GB, E_C, E_LJ) and analytic dE/dx [N,3], dE/dq [N], dE/drho [N]."""
    gb = gb or obc2()
    xyz = _f64(xyz).reshape(-1)
    n = xyz.size // 3
    E, gx, gq, gr = np.zeros(3), np.zeros(3 * n), np.zeros(n), np.zeros(n)
    lib().orc_gradient(n, xyz, _f64(q), _f64(rho), _f64(scr), _f64(sig), _f64(eps),
                       C.byref(gb), E, gx, gq, gr)
    return E, gx.reshape(n, 3), gq, gr


def energy(xyz, q, rho, scr, sig, eps, gb=None):
    """Total (E_GB, E_C, E_LJ) of one system, Born radii computed from xyz."""
    _, R, _ = born(xyz, rho, scr, gb)
    return energy_at_R(xyz, q, R, sig, eps, gb)


def tether(xyz, x0, k):
    xyz = _f64(xyz).reshape(-1)
    g = np.zeros_like(xyz)
    e = lib().orc_tether(xyz.size // 3, xyz, _f64(x0).reshape(-1), float(k), g)
    return e, g.reshape(-1, 3)


def eval_batch(atom_off, xyz, q, rho, scr, sig, eps, gb=None):
    """Per-replica energies [R,3] and gradients for a flat batch of replicas."""
    off = np.asarray(atom_off)
    n_rep = off.size - 1
    E = np.zeros((n_rep, 3))
    gx = np.zeros((off[-1], 3))
    gq = np.zeros(off[-1])
    gr = np.zeros(off[-1])
    for r in range(n_rep):
        a, b = off[r], off[r + 1]
        E[r], gx[a:b], gq[a:b], gr[a:b] = gradient(xyz[a:b], q[a:b], rho[a:b], scr[a:b],
                                                   sig[a:b], eps[a:b], gb)
    return E, gx, gq, gr


def born_batch(atom_off, xyz, rho, scr, gb=None):
    off = np.asarray(atom_off)
    psi = np.zeros(off[-1]); R = np.zeros(off[-1]); d = np.zeros(off[-1])
    for r in range(off.size - 1):
        a, b = off[r], off[r + 1]
        psi[a:b], R[a:b], d[a:b] = born(xyz[a:b], rho[a:b], scr[a:b], gb)
    return psi, R, d


# ------------------------------------------------------------------ MD / MC / REMD
@dataclass
class _Keep:
    """Holds the numpy arrays a ctypes struct points into."""
    arrays: list


def _ptr(a, ct):
    return a.ctypes.data_as(_P(ct))


def make_md(sysd: dict, gb=None, seed=0, eps_mode=0):
    """Build (cfg, state, keep) ctypes structures from a synthetic-system dict
    (the fields produced by the generator, see ``tests/conftest.py``).  The
    state arrays are float64/int32 copies owned by ``keep``."""
    gb = gb or obc2()
    keep = []

    def f(a):
        a = _f64(a).copy(); keep.append(a); return a

    def i(a):
        a = _i32(a).copy(); keep.append(a); return a

    def ll(n):
        a = np.zeros(max(n, 1), dtype=np.int64); keep.append(a); return a

    cfg = MDCfg()
    off = i(sysd["atom_off"])
    cfg.n_rep = off.size - 1
    cfg.atom_off = _ptr(off, C.c_int)
    cfg.n_sites = int(sysd["n_sites"])
    cfg.max_states = int(sysd["max_states"])
    for name in ("rep_site_off", "site_off", "site_atoms", "site_type", "n_states",
                 "state_nH", "state_ne"):
        setattr(cfg, name, _ptr(i(sysd[name]), C.c_int))
    for name in ("state_q", "G_ref", "ref_value"):
        setattr(cfg, name, _ptr(f(sysd[name]), C.c_double))
    H_scale = np.asarray(sysd.get("H_scale", [1.0]), np.float64)
    cfg.n_inst, cfg.nE, cfg.npH, cfg.nT, cfg.nHam = (int(sysd["n_inst"]), len(sysd["E_vals"]),
                                                     len(sysd["pH_vals"]), len(sysd["T_vals"]),
                                                     H_scale.size)
    for name in ("E_vals", "pH_vals", "T_vals"):
        setattr(cfg, name, _ptr(f(sysd[name]), C.c_double))
    cfg.H_scale = _ptr(f(H_scale), C.c_double)
    order = list(sysd["dim_order"])
    cfg.n_dims = len(order)
    for k in range(4):
        cfg.dim_order[k] = order[k] if k < len(order) else 0
    for name, key in (("rho", "rho"), ("scr", "screen"), ("sig", "sigma"), ("eps", "eps"),
                      ("mass", "mass")):
        setattr(cfg, name, _ptr(f(sysd[key]), C.c_double))
    cfg.x0 = _ptr(f(np.asarray(sysd["x0"]).reshape(-1)), C.c_double)
    cfg.gb = gb
    cfg.k_tether = float(sysd["k_tether"])
    cfg.dt = float(sysd["dt"])
    cfg.gamma_ps = float(sysd["gamma_ps"])
    cfg.mc_every = int(sysd["mc_every"])
    cfg.ex_every = int(sysd["ex_every"])
    cfg.eps_mode = int(eps_mode)
    cfg.seed = int(seed)

    n_tot = int(off[-1])
    st = MDState()
    arrs = {
        "xyz": f(np.asarray(sysd["xyz"]).reshape(-1)),
        "v": f(np.asarray(sysd.get("v", np.zeros((n_tot, 3)))).reshape(-1)),
        "q": f(sysd["q"]),
        "F": f(np.zeros(3 * n_tot)),
        "E": f(np.zeros(4 * cfg.n_rep)),
        "site_state": i(sysd["site_state"]),
        "target_idx": i(np.asarray(sysd["target_idx"]).reshape(-1)),
        "grid_rep": i(sysd["grid_rep"]),
        "mc_att": ll(cfg.n_sites), "mc_acc": ll(cfg.n_sites),
        "ex_att": ll(4 * cfg.n_rep),
        "ex_acc": ll(4 * cfg.n_rep),
    }
    for k, a in arrs.items():
        ct = C.c_double if a.dtype == np.float64 else (C.c_int if a.dtype == np.int32 else C.c_longlong)
        setattr(st, k, _ptr(a, ct))
    return cfg, st, arrs, keep


def md_run(cfg, st, step0: int, n_steps: int, init_forces: bool):
    return lib().orc_md_run(C.byref(cfg), C.byref(st), int(step0), int(n_steps), int(init_forces))


def replica_counts(cfg, site_state, target_idx, E4):
    n = cfg.n_rep
    nH, ne, ep = np.zeros(n, np.int32), np.zeros(n, np.int32), np.zeros(n)
    a, b, c = C.c_int(), C.c_int(), C.c_double()
    ss, ti, e4 = _i32(site_state), _i32(np.asarray(target_idx).reshape(-1)), _f64(E4).reshape(-1)
    for r in range(n):
        lib().orc_replica_counts(C.byref(cfg), ss, ti, e4, r, C.byref(a), C.byref(b), C.byref(c))
        nH[r], ne[r], ep[r] = a.value, b.value, c.value
    return nH, ne, ep


def exchange(cfg, attempt, nH, ne, epsT, target_idx, grid_rep, E4=None):
    """One exchange attempt; E4 [n_rep, 4] (GB, Coulomb, LJ, tether) is read by
    Hamiltonian attempts.  Returns (target_idx, grid_rep, vscale, att, acc)."""
    ti = _i32(np.asarray(target_idx).reshape(-1)).copy()
    gr = _i32(grid_rep).copy()
    vs = np.ones(cfg.n_rep)
    GT = cfg.n_inst * cfg.nE * cfg.npH * cfg.nT * cfg.nHam
    att = np.zeros(4 * GT, dtype=np.int64)
    acc = np.zeros(4 * GT, dtype=np.int64)
    e4 = _f64(np.zeros((cfg.n_rep, 4)) if E4 is None else E4).reshape(-1)
    lib().orc_exchange(C.byref(cfg), int(attempt), _i32(nH), _i32(ne), _f64(epsT), e4, ti, gr, vs,
                       att.ctypes.data_as(_P(C.c_longlong)), acc.ctypes.data_as(_P(C.c_longlong)))
    return ti.reshape(-1, 4), gr, vs, att, acc
