"""GPU-test helpers: run the HIP path through the C ABI on a generator batch
and fetch results as float64 numpy arrays for comparison with the oracle."""
import os

import numpy as np
import torch

FX_F = 2.0 ** -40
FX_E = 2.0 ** -32

# Tolerances (the contract of the FP32-pair / fixed-point path against FP64):
E_TOL = 1e-6          # relative, total energy and E_GB
F_TOL = 1e-5          # RMS-relative force error per replica
R_TOL = 2e-6          # relative Born radius (FP32 storage of R: 6e-8 ulp)
F_ATOM_TOL = 1e-4     # worst single atom: |F_gpu,i - F64,i| over the replica's RMS force
DE_TOL = 1e-6         # titration dE: |dE_gpu - dE64| over the sum of the absolute values
                      # of the incremental form's terms (FP32 terms, each within a few
                      # 2^-24 relative, added in FP32 partials and 64-bit fixed point)

# worst value of each error seen per test, printed at the end of the run
MEASURED = {}


def note(quantity, value):
    test = os.environ.get("PYTEST_CURRENT_TEST", "?").split(" ")[0]
    key = (test, quantity)
    MEASURED[key] = max(MEASURED.get(key, 0.0), float(value))


def to_dev(b):
    from paper_1809_07726_amd.gb import DeviceBatch
    return DeviceBatch.from_numpy(b)


def soa_to_aos(x, n):
    return np.asarray(x, dtype=np.float64).reshape(3, n).T


def gpu_eval(b, grad_q=False, grad_rho=False, blocking=None, launch=None, params=None, split=None):
    """Born radii, energies and gradients of every replica on the GPU."""
    from paper_1809_07726_amd.gb import Context
    ctx = Context(b["atom_off"], params)
    if split:
        ctx.set_split(split)
    if blocking:
        ctx.set_blocking(*blocking)
    if launch:
        ctx.set_launch(*launch)
    d = to_dev(b)
    t = d.t
    R, dR, psi = ctx.born_radii(t["xyz"], t["rho"], t["screen"])
    f, e, dq, dr = ctx.energy_forces(t["xyz"], t["q"], t["rho"], t["screen"], t["sigma"], t["eps"],
                                     R, dR, psi, grad_q=grad_q, grad_rho=grad_rho)
    E = ctx.energies(e)
    ctx.check()
    N = ctx.n_atoms
    out = {"R": R.cpu().double().numpy(), "psi": psi.cpu().numpy(),
           "F": soa_to_aos(f.cpu().numpy() * FX_F, N), "F_fx": f.cpu().numpy(),
           "E": E.cpu().numpy(), "E_fx": e.cpu().numpy()}
    if grad_q:
        out["dEdq"] = dq.cpu().numpy() * FX_F
    if grad_rho:
        out["dEdrho"] = dr.cpu().numpy() * FX_F
    ctx.close()
    return out


def rms_rel(a, b):
    return float(np.sqrt(((a - b) ** 2).sum() / (b ** 2).sum()))


def worst_rel(a, b):
    """Largest per-row error norm over the RMS row norm of the reference (rows
    are atoms: [N, 3] forces, or [N] per-atom derivatives)."""
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    if a.ndim == 1:
        a, b = a[:, None], b[:, None]
    d = np.sqrt(((a - b) ** 2).sum(1))
    return float(d.max() / np.sqrt((b ** 2).sum(1).mean()))


def check_per_atom(g, o, what="force"):
    """RMS-relative and worst-atom error of per-atom vectors against the FP64
    oracle, recorded and held to F_TOL and F_ATOM_TOL."""
    e_rms, e_atom = rms_rel(g, o), worst_rel(g, o)
    note(what + " rms-rel", e_rms)
    note(what + " worst atom / rms", e_atom)
    assert e_rms < F_TOL, (what, e_rms)
    assert e_atom < F_ATOM_TOL, (what, e_atom)


def check_energy(Eg, Eo):
    """Per-replica energies (GPU row: GB, C, LJ, tether, total; oracle: GB, C,
    LJ): total and E_GB to E_TOL relative, C and LJ to E_TOL of sum |E|."""
    tot = Eo.sum()
    err_t, err_gb = abs(Eg[4] - tot), abs(Eg[0] - Eo[0])
    if tot != 0.0:
        note("energy rel", err_t / abs(tot))
    if Eo[0] != 0.0:
        note("E_GB rel", err_gb / abs(Eo[0]))
    assert err_t <= E_TOL * abs(tot) and err_gb <= E_TOL * abs(Eo[0]), (Eg, Eo)
    assert abs(Eg[1] - Eo[1]) <= E_TOL * abs(Eo).sum()
    assert abs(Eg[2] - Eo[2]) <= E_TOL * abs(Eo).sum()


def check_delta_e(dE, ref, scale, what="titration dE"):
    """A titration energy change against the oracle's: the error over the
    absolute-term sum `scale` held to DE_TOL; the error relative to |dE|
    itself is recorded too."""
    err = abs(dE - ref)
    note(what + " err / term-sum", err / scale)
    note(what + " err / |dE|", err / max(abs(ref), 1e-300))
    assert err <= DE_TOL * scale, (dE, ref, scale)


def clear_cutoffs(b, cut0, rgb0, gap=5e-5):
    """cut and rgbmax near the requested values, moved by steps of 0.013 A until
    no pair of any replica lies within gap of either: a pair within FP32
    rounding of a cutoff (about 1e-5 A at 10 A) may be counted on one side and
    not on the other."""
    off = b["atom_off"]
    r = []
    for k in range(off.size - 1):
        x = b["xyz"][off[k]:off[k + 1]].astype(np.float64)
        d = np.sqrt(((x[:, None] - x[None]) ** 2).sum(-1))
        r.append(d[np.triu_indices(len(x), 1)])
    r = np.concatenate(r)
    pick = lambda c0: next(c for c in c0 + 0.013 * np.arange(200) if np.abs(r - c).min() > gap)
    return pick(cut0), pick(rgb0)
