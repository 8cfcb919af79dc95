"""GPU-test helpers: run the HIP path through the C ABI on a generator batch
and fetch results as float64 numpy arrays for comparison with the oracle."""
import numpy as np
import torch

FX_F = 2.0 ** -40
FX_E = 2.0 ** -32

# Tolerances (the contract of the FP32-pair / fixed-point path against FP64):
E_TOL = 1e-6          # relative, total energy and E_GB
F_TOL = 1e-5          # RMS-relative force error per replica
R_TOL = 2e-6          # relative Born radius (FP32 storage of R: 6e-8 ulp)


def to_dev(b):
    from paper_1809_07726_amd.gb import DeviceBatch
    return DeviceBatch.from_numpy(b)


def soa_to_aos(x, n):
    return np.asarray(x, dtype=np.float64).reshape(3, n).T


def gpu_eval(b, grad_q=False, grad_rho=False, blocking=None, launch=None, params=None):
    """Born radii, energies and gradients of every replica on the GPU."""
    from paper_1809_07726_amd.gb import Context
    ctx = Context(b["atom_off"], params)
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
