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


def test_grid_validation_of_the_hamiltonian_dimension():
    """md_step and remd_exchange reject a grid whose sizes do not multiply to
    the replica count, nHam > 1 without scales, and dimension codes out of
    range, before launching anything."""
    import torch
    import paper_1809_07726_amd._capi as A
    from paper_1809_07726_amd import synth
    from paper_1809_07726_amd.gb import MD, Context, DeviceBatch
    base = synth.draw_system(32, 5, 0, 0)
    base["sites"] = []
    b = synth.assemble([base], 4, (-0.2,), (7.0,), (300.0, 320.0), (synth.DIM_T, synth.DIM_H),
                       H_scale=(1.0, 0.9), mc_every=0, ex_every=1)
    ctx = Context(b["atom_off"])
    d = DeviceBatch.from_numpy(b)
    md = MD(ctx, d, b, seed=1)
    md.run(1, init_forces=True)                       # the valid grid runs
    g = md.pr.grid
    bad = []
    saved = (g.nHam, g.H_scale, g.n_dims, g.dim_order[1])
    g.H_scale = None
    bad.append(A.lib.md_step(ctx.h, C.byref(md.st), C.byref(md.pr), 1, 1, 1, 0, A.stream_handle()))
    g.H_scale = saved[1]
    g.nHam = 3
    bad.append(A.lib.md_step(ctx.h, C.byref(md.st), C.byref(md.pr), 1, 1, 1, 0, A.stream_handle()))
    g.nHam = saved[0]
    g.dim_order[1] = 4
    bad.append(A.lib.md_step(ctx.h, C.byref(md.st), C.byref(md.pr), 1, 1, 1, 0, A.stream_handle()))
    g.dim_order[1] = saved[3]
    g.n_dims = 5
    bad.append(A.lib.md_step(ctx.h, C.byref(md.st), C.byref(md.pr), 1, 1, 1, 0, A.stream_handle()))
    g.n_dims = saved[2]
    assert bad == [A.GBR_E_INVAL] * 4, bad
    R = ctx.n_rep
    z = torch.zeros(R, dtype=torch.int32, device="cuda")
    with pytest.raises(A.GBRError):                    # an H grid needs the nonbonded energies
        ctx.remd_exchange(g, 1, z, z, torch.zeros(R, dtype=torch.float64, device="cuda"),
                          d.t["target_idx"], d.t["grid_rep"], seed=1)
    md.run(1)                                         # and the context still works
    torch.cuda.synchronize()
    assert _check(ctx) == (A.GBR_OK, 0)
    ctx.close()
