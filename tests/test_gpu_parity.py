"""Parity of the HIP path (through the C ABI) with the FP64 oracle on the same
seeded inputs: Born radii, energies and forces, titration energy changes;
determinism; every register-blocking variant; ragged and uneven batches."""
import numpy as np
import pytest

import oracle
from gpu_common import R_TOL, check_delta_e, check_energy, check_per_atom, clear_cutoffs, gpu_eval, note
from paper_1809_07726_amd import synth

pytestmark = pytest.mark.gpu


def _oracle_batch(b, grads=True, gb=None):
    off = b["atom_off"]
    E, gx, gq, gr = oracle.eval_batch(off, b["xyz"], b["q"], b["rho"], b["screen"], b["sigma"], b["eps"], gb)
    psi, R, _ = oracle.born_batch(off, b["xyz"], b["rho"], b["screen"], gb)
    return {"E": E, "F": -gx, "dEdq": gq, "dEdrho": gr, "R": R, "psi": psi}


def _check(b, g, o, grads=False):
    off = b["atom_off"]
    rel_R = np.abs(g["R"] / o["R"] - 1).max()
    note("Born radius rel", rel_R)
    assert rel_R < R_TOL
    for r in range(off.size - 1):
        a, c = off[r], off[r + 1]
        check_energy(g["E"][r], o["E"][r])
        if c - a > 1:
            check_per_atom(g["F"][a:c], o["F"][a:c])
            if grads:
                check_per_atom(g["dEdq"][a:c], o["dEdq"][a:c], "dE/dq")
                check_per_atom(g["dEdrho"][a:c], o["dEdrho"][a:c], "dE/drho")


def test_c0_single_replica():
    b = synth.make_config(0)
    _check(b, gpu_eval(b, True, True), _oracle_batch(b), grads=True)


def test_replicas_with_distinct_geometry():
    """Replicas of the 1024-atom E,T,pH system with independent jitter, so a
    replica-indexing mistake cannot hide behind identical copies."""
    b = synth.make_config(2, n_rep=6, per_replica_jitter=True)
    _check(b, gpu_eval(b), _oracle_batch(b))


def test_ragged_uneven_replicas():
    """Replica sizes that are not multiples of the 64-atom tile, including a
    single atom and sizes smaller than one tile."""
    sizes = [1, 2, 37, 64, 65, 100, 257, 500, 700]
    systems = [synth.draw_system(n, 500 + n, 1 if n >= 16 else 0, 1 if n >= 16 else 0) for n in sizes]
    b = synth.assemble(systems, 1, (-0.2,), (7.0,), (300.0,), (0,))
    _check(b, gpu_eval(b, True, True), _oracle_batch(b), grads=True)


@pytest.mark.parametrize("ni", [1, 2, 4, 8])
def test_every_register_blocking(ni):
    b = synth.make_config(1, n_atoms=700, n_rep=2, per_replica_jitter=True)
    _check(b, gpu_eval(b, True, True, blocking=(ni, ni, ni)), _oracle_batch(b), grads=True)


@pytest.mark.parametrize("ni", [1, 2, 4])
def test_every_block_item_halved_matches_oracle(ni):
    """Split level 1 (every block item run as two halves) on ragged replicas,
    with the radius and charge gradients, against the oracle."""
    sizes = [1, 37, 64, 65, 300, 700, 1300]
    systems = [synth.draw_system(n, 600 + n, 1 if n >= 16 else 0, 1 if n >= 16 else 0) for n in sizes]
    b = synth.assemble(systems, 1, (-0.2,), (7.0,), (300.0,), (0,))
    # items hold their partials in FP32 until their flush, so halving changes
    # the rounding, not the sum: held to the oracle, not to the default level
    _check(b, gpu_eval(b, True, True, blocking=(ni, ni, ni), split=1), _oracle_batch(b), grads=True)


@pytest.mark.parametrize("ni", [1, 2])
def test_launch_shapes_are_bitwise_identical(ni):
    """One wavefront per workgroup or four, few or many workgroups per CU: each
    item's partial sums do not depend on which wavefront runs it and the
    fixed-point atomics are order-independent, so every shape gives the same
    bits; one of them is checked against the oracle."""
    b = synth.make_config(1, n_atoms=700, n_rep=3, per_replica_jitter=True)
    ref = None
    for shape in ((1, 1), (1, 32), (2, 32), (4, 8), (4, 32)):
        g = gpu_eval(b, True, True, blocking=(ni, ni, ni), launch=shape)
        if ref is None:
            ref = g
            _check(b, g, _oracle_batch(b), grads=True)
            continue
        for k in ("F_fx", "E_fx", "R", "dEdq", "dEdrho"):
            assert np.array_equal(g[k], ref[k]), (shape, k)


def test_bitwise_reproducible_and_newton_balanced():
    b = synth.make_config(2, n_rep=4, per_replica_jitter=True)
    g1 = gpu_eval(b, True, True)
    g2 = gpu_eval(b, True, True)
    assert np.array_equal(g1["F_fx"], g2["F_fx"])
    assert np.array_equal(g1["E_fx"], g2["E_fx"])
    assert np.array_equal(g1["R"], g2["R"])
    # Newton's third law: each pair force enters the i-side and the j-side FP32
    # partial sums, which round differently, so the net force vanishes only to
    # a few FP32 ulps of the summed magnitudes (the oracle's is zero to FP64).
    off = b["atom_off"]
    for r in range(off.size - 1):
        F = g1["F"][off[r]:off[r + 1]]
        assert np.abs(F.sum(0)).max() <= 2e-8 * np.abs(F).sum()


@pytest.mark.parametrize("n_atoms,n_rep", [(None, 4), (5000, 2)])
def test_titration_delta_e_matches_oracle(n_atoms, n_rep):
    """Every site's state-1 candidate against the oracle's direct difference;
    5,000-atom replicas split the sum over the replica's atoms into three
    chunks."""
    from paper_1809_07726_amd.gb import Context
    from gpu_common import to_dev
    import torch
    b = synth.make_config(1, n_atoms=n_atoms, n_rep=n_rep, per_replica_jitter=True)
    d = to_dev(b)
    ctx = Context(b["atom_off"])
    t = d.t
    R, _, _ = ctx.born_radii(t["xyz"], t["rho"], t["screen"])
    cand = np.array([(s, 1) for s in range(b["n_sites"])], np.int32).reshape(-1)
    dE = ctx.titration_delta_e(t["xyz"], t["q"], R, d, torch.as_tensor(cand)).cpu().numpy()
    ctx.check()
    off = b["atom_off"]
    ms = b["max_states"]
    for s in range(b["n_sites"]):
        r = int(np.searchsorted(off, b["site_atoms"][b["site_off"][s]], side="right") - 1)
        a0, a1 = off[r], off[r + 1]
        x = b["xyz"][a0:a1]
        _, Ro, _ = oracle.born(x, b["rho"][a0:a1], b["screen"][a0:a1])
        sl = slice(b["site_off"][s], b["site_off"][s + 1])
        idx = b["site_atoms"][sl] - a0
        qn = b["state_q"].reshape(-1, ms)[sl, 1]
        ref = oracle.delta_e(x, b["q"][a0:a1], Ro, idx, qn)
        check_delta_e(dE[s], ref, oracle.delta_e_abs_scale(x, b["q"][a0:a1], Ro, idx, qn))


def test_titration_delta_e_for_every_state_of_three_state_sites():
    """pH sites with a third state: the candidate (site, state) energy change
    for states 1 and 2 of every pH site (and state 1 of every redox site)
    against the oracle's direct difference."""
    from paper_1809_07726_amd.gb import Context
    from gpu_common import to_dev
    from common import with_diprotic_ph_sites
    import torch
    b = with_diprotic_ph_sites(synth.make_config(1, n_rep=3, per_replica_jitter=True))
    d = to_dev(b)
    ctx = Context(b["atom_off"])
    t = d.t
    R, _, _ = ctx.born_radii(t["xyz"], t["rho"], t["screen"])
    pairs = [(s, k) for s in range(b["n_sites"]) for k in range(1, int(b["n_states"][s]))]
    assert any(k == 2 for _, k in pairs)
    cand = np.array(pairs, np.int32).reshape(-1)
    dE = ctx.titration_delta_e(t["xyz"], t["q"], R, d, torch.as_tensor(cand)).cpu().numpy()
    ctx.check()
    ctx.close()
    off = b["atom_off"]
    ms = b["max_states"]
    for i, (s, k) in enumerate(pairs):
        r = int(np.searchsorted(off, b["site_atoms"][b["site_off"][s]], side="right") - 1)
        a0, a1 = off[r], off[r + 1]
        x = b["xyz"][a0:a1]
        _, Ro, _ = oracle.born(x, b["rho"][a0:a1], b["screen"][a0:a1])
        sl = slice(b["site_off"][s], b["site_off"][s + 1])
        idx = b["site_atoms"][sl] - a0
        qn = b["state_q"].reshape(-1, ms)[sl, k]
        ref = oracle.delta_e(x, b["q"][a0:a1], Ro, idx, qn)
        check_delta_e(dE[i], ref, oracle.delta_e_abs_scale(x, b["q"][a0:a1], Ro, idx, qn))


# --------------------------- salt screening and pair cutoffs (kappa, cut, rgbmax)
@pytest.mark.parametrize("ni", [1, 2, 4, 8])
@pytest.mark.parametrize("kappa,cut,rgb", [(0.15, 10.0, 12.0), (0.1, 0.0, 0.0), (0.0, 9.0, 0.0),
                                           (0.0, 0.0, 8.0)])
def test_salt_and_cutoffs_match_oracle(ni, kappa, cut, rgb):
    """Energies, forces, dE/dq and dE/drho with salt and with either cutoff
    alone or both, for every register blocking, against the oracle with the
    same settings; and the settings do change the result."""
    import paper_1809_07726_amd._capi as A
    b = synth.make_config(1, n_atoms=700, n_rep=2, per_replica_jitter=True)
    if cut or rgb:
        c, g_ = clear_cutoffs(b, cut or 9.0, rgb or 9.0)
        cut, rgb = (c if cut else 0.0), (g_ if rgb else 0.0)
    P = A.obc2(kappa=kappa, cut=cut, rgbmax=rgb)
    G = oracle.obc2(kappa=kappa, cut=cut, rgbmax=rgb)
    g = gpu_eval(b, True, True, blocking=(ni, ni, ni), params=P)
    o = _oracle_batch(b, gb=G)
    _check(b, g, o, grads=True)
    plain = _oracle_batch(b)
    assert np.abs(plain["E"] - o["E"]).max() > 1e-3


@pytest.mark.parametrize("ni", [1, 2, 4, 8])
def test_ragged_uneven_replicas_with_packed_cutoff_lists(ni):
    """Replica sizes from one atom to several 64-atom tiles (ragged tails,
    blocks with and without tiles after them) in one batch with salt and both
    cutoffs, so that every blocking's packed lists span replicas of every
    shape."""
    import paper_1809_07726_amd._capi as A
    sizes = [1, 2, 37, 64, 65, 130, 257, 520, 700, 1300]
    systems = [synth.draw_system(n, 900 + n, 1 if n >= 16 else 0, 1 if n >= 16 else 0, blocked=n >= 64)
               for n in sizes]
    b = synth.assemble(systems, 1, (-0.2,), (7.0,), (300.0,), (0,))
    cut, rgb = clear_cutoffs(b, 8.0, 10.0)
    P = A.obc2(kappa=0.1, cut=cut, rgbmax=rgb)
    G = oracle.obc2(kappa=0.1, cut=cut, rgbmax=rgb)
    _check(b, gpu_eval(b, True, True, blocking=(ni, ni, ni), params=P), _oracle_batch(b, gb=G), grads=True)


@pytest.mark.parametrize("n_atoms,n_rep", [(None, 3), (5000, 2)])
def test_titration_delta_e_with_salt_and_cutoff_matches_oracle(n_atoms, n_rep):
    """Salt and the pair cutoff in the titration sums, with 1,024-atom
    replicas (one chunk) and 5,000-atom replicas (three chunks)."""
    import paper_1809_07726_amd._capi as A
    import torch
    from paper_1809_07726_amd.gb import Context
    from gpu_common import to_dev
    b = synth.make_config(1, n_atoms=n_atoms, n_rep=n_rep, per_replica_jitter=True)
    if n_atoms is None:
        cut, rgb = clear_cutoffs(b, 9.0, 11.0)
    else:
        # many pairs: only the site atoms' distances decide the titration sums,
        # and the Born radii are left without a cutoff
        off = b["atom_off"]
        r = []
        for s_ in range(b["n_sites"]):
            rr = int(np.searchsorted(off, b["site_atoms"][b["site_off"][s_]], side="right") - 1)
            xs = b["xyz"][b["site_atoms"][b["site_off"][s_]:b["site_off"][s_ + 1]]].astype(np.float64)
            xa = b["xyz"][off[rr]:off[rr + 1]].astype(np.float64)
            r.append(np.sqrt(((xs[:, None] - xa[None]) ** 2).sum(-1)).ravel())
        r = np.concatenate(r)
        cut = next(c for c in 9.0 + 0.013 * np.arange(200) if np.abs(r - c).min() > 5e-5)
        rgb = 0.0
    P = A.obc2(kappa=0.2, cut=cut, rgbmax=rgb)
    G = oracle.obc2(kappa=0.2, cut=cut, rgbmax=rgb)
    d = to_dev(b)
    ctx = Context(b["atom_off"], P)
    t = d.t
    R, _, _ = ctx.born_radii(t["xyz"], t["rho"], t["screen"])
    cand = np.array([(s, 1) for s in range(b["n_sites"])], np.int32).reshape(-1)
    dE = ctx.titration_delta_e(t["xyz"], t["q"], R, d, torch.as_tensor(cand)).cpu().numpy()
    ctx.check()
    ctx.close()
    off = b["atom_off"]
    ms = b["max_states"]
    for s in range(b["n_sites"]):
        r = int(np.searchsorted(off, b["site_atoms"][b["site_off"][s]], side="right") - 1)
        a0, a1 = off[r], off[r + 1]
        x = b["xyz"][a0:a1]
        _, Ro, _ = oracle.born(x, b["rho"][a0:a1], b["screen"][a0:a1], G)
        sl = slice(b["site_off"][s], b["site_off"][s + 1])
        idx = b["site_atoms"][sl] - a0
        qn = b["state_q"].reshape(-1, ms)[sl, 1]
        ref = oracle.delta_e(x, b["q"][a0:a1], Ro, idx, qn, G)
        check_delta_e(dE[s], ref, oracle.delta_e_abs_scale(x, b["q"][a0:a1], Ro, idx, qn, G))
