"""The device error word: a non-finite or out-of-range value met by the pair
kernels' fixed-point conversions is reported by gbr_check (GBR_E_NUMERIC with
the GBR_ERR_* bits) instead of being summed silently; the check that reports
it clears it, and the next clean evaluation reports nothing."""
import ctypes as C

import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def setup():
    import torch
    from paper_1809_07726_amd import synth
    from paper_1809_07726_amd.gb import Context, DeviceBatch
    assert torch.cuda.is_available()
    b = synth.make_config(1, n_atoms=300, n_rep=2)
    ctx = Context(b["atom_off"])
    d = DeviceBatch.from_numpy(b)
    yield ctx, d.t
    ctx.close()


def _eval(ctx, t):
    R, dR, psi = ctx.born_radii(t["xyz"], t["rho"], t["screen"])
    ctx.energy_forces(t["xyz"], t["q"], t["rho"], t["screen"], t["sigma"], t["eps"], R, dR, psi)


def _check(ctx):
    import paper_1809_07726_amd._capi as A
    bits = C.c_uint32()
    rc = A.lib.gbr_check(ctx.h, A.stream_handle(), C.byref(bits))
    return rc, bits.value


def test_clean_evaluation_reports_nothing(setup):
    import paper_1809_07726_amd._capi as A
    ctx, t = setup
    _eval(ctx, t)
    assert _check(ctx) == (A.GBR_OK, 0)


def test_nonfinite_coordinate_is_reported_then_cleared(setup):
    import paper_1809_07726_amd._capi as A
    ctx, t = setup
    x = t["xyz"].clone()
    x[5] = float("nan")
    print("case: NaN x coordinate of atom 5", flush=True)
    _eval(ctx, {**t, "xyz": x})
    rc, bits = _check(ctx)
    assert rc == A.GBR_E_NUMERIC and bits & A.ERR_NONFINITE, (rc, bits)
    assert _check(ctx) == (A.GBR_OK, 0)
    _eval(ctx, t)
    assert _check(ctx) == (A.GBR_OK, 0)


def test_saturating_charge_sets_the_overflow_bit(setup):
    import paper_1809_07726_amd._capi as A
    ctx, t = setup
    q = t["q"].clone()
    q[7] = 1.0e12        # finite, but its pair energies and forces exceed 2^62 fixed-point units
    print("case: charge 1e12 on atom 7", flush=True)
    _eval(ctx, {**t, "q": q})
    rc, bits = _check(ctx)
    assert rc == A.GBR_E_NUMERIC and bits & A.ERR_OVERFLOW and not bits & A.ERR_NONFINITE, (rc, bits)
    assert _check(ctx) == (A.GBR_OK, 0)
