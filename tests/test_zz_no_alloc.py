"""gb_born_radii_noalloc, the entry point for callers that cannot allocate
device memory, against gb_born_radii: two calls in a row on one device (the
second with a smaller batch, so a stale sum left in the shared static array
would show), with and without the descreening cutoff; the host rejects a
batch beyond the array's size, and a replica larger than max_atoms is
reported in the error word."""
import ctypes as C

import numpy as np
import pytest
import torch

from gpu_common import R_TOL, clear_cutoffs, note, to_dev
from paper_1809_07726_amd import synth

pytestmark = pytest.mark.gpu


def _batch(sizes, seed0):
    systems = [synth.draw_system(n, seed0 + n, 1 if n >= 16 else 0, 1 if n >= 16 else 0) for n in sizes]
    return synth.assemble(systems, 1, (-0.2,), (7.0,), (300.0,), (0,))


def _noalloc(b, P, max_atoms=None):
    import paper_1809_07726_amd._capi as A
    t = to_dev(b).t
    off = torch.as_tensor(np.asarray(b["atom_off"], np.int32), device="cuda")
    N = int(b["atom_off"][-1])
    mx = int(np.diff(b["atom_off"]).max()) if max_atoms is None else max_atoms
    R = torch.full((N,), float("nan"), dtype=torch.float32, device="cuda")
    dR = torch.full((N,), float("nan"), dtype=torch.float32, device="cuda")
    psi = torch.full((N,), float("nan"), dtype=torch.float64, device="cuda")
    err = torch.zeros(1, dtype=torch.int32, device="cuda")
    print(f"gb_born_radii_noalloc: {b['n_rep']} replicas, {N} atoms, max_atoms {mx}, rgbmax {P.rgbmax}",
          flush=True)
    A.check(A.lib.gb_born_radii_noalloc(C.byref(P), int(b["n_rep"]), off.data_ptr(), N, mx,
                                        A.ptr(t["xyz"]), A.ptr(t["rho"]), A.ptr(t["screen"]),
                                        R.data_ptr(), dR.data_ptr(), psi.data_ptr(), err.data_ptr(),
                                        A.stream_handle()))
    torch.cuda.synchronize()
    return (R.cpu().double().numpy(), dR.cpu().double().numpy(), psi.cpu().numpy(), int(err.item()))


def _with_context(b, P):
    from paper_1809_07726_amd.gb import Context
    ctx = Context(b["atom_off"], P)
    t = to_dev(b).t
    R, dR, psi = ctx.born_radii(t["xyz"], t["rho"], t["screen"])
    ctx.check()
    out = (R.cpu().double().numpy(), dR.cpu().double().numpy(), psi.cpu().numpy())
    ctx.close()
    return out


def _compare(b, P):
    R, dR, psi, err = _noalloc(b, P)
    assert err == 0
    Rc, dRc, psic = _with_context(b, P)
    rel_R = np.abs(R / Rc - 1).max()
    note("noalloc R rel", rel_R)
    assert rel_R < R_TOL
    assert np.abs(psi - psic).max() <= 1e-6 * np.abs(psic).max()
    assert np.abs(dR - dRc).max() <= 1e-5 * np.abs(dRc).max()


@pytest.mark.parametrize("cutoff", [False, True])
def test_noalloc_born_radii_match_the_context_path_on_two_calls(cutoff):
    import paper_1809_07726_amd._capi as A
    big = _batch([1, 37, 300, 700, 1300], 700)
    small = _batch([64, 65, 200], 800)
    rgb = clear_cutoffs(big, 9.0, 9.0)[1] if cutoff else 0.0
    if cutoff:
        rgb = clear_cutoffs(small, rgb, rgb)[1]
    P = A.obc2(rgbmax=rgb)
    _compare(big, P)
    _compare(small, P)


def test_noalloc_rejects_oversize_and_reports_layout():
    import paper_1809_07726_amd._capi as A
    P = A.obc2()
    dummy = torch.zeros(8, dtype=torch.float32, device="cuda")
    off = torch.zeros(2, dtype=torch.int32, device="cuda")
    n_big = A.NOALLOC_MAX_ATOMS + 1
    p = dummy.data_ptr()
    rc = A.lib.gb_born_radii_noalloc(C.byref(P), 1, off.data_ptr(), n_big, n_big, p, p, p, p, p, None, p,
                                     A.stream_handle())
    assert rc == A.GBR_E_INVAL and b"static scratch" in A.lib.gbr_last_error()
    # max_atoms below the largest replica: that replica is skipped and flagged,
    # the others stay exact
    b = _batch([100, 300, 90], 900)
    R, dR, psi, err = _noalloc(b, P, max_atoms=128)
    assert err & A.ERR_LAYOUT
    Rc, _, _ = _with_context(b, P)
    off_h = b["atom_off"]
    for r in (0, 2):
        sl = slice(off_h[r], off_h[r + 1])
        assert np.abs(R[sl] / Rc[sl] - 1).max() < R_TOL
