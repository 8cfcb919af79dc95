"""The adjoint behind torch.autograd (dE/dx, dE/dq, dE/drho) against the FP64
oracle's analytic gradient, and the batched evaluation at the full workload
sizes: sampled replicas against the oracle, properties that hold at any size
for the rest (finite energies, vanishing net force, run-to-run identity)."""
import numpy as np
import pytest
import torch

import oracle
from gpu_common import (check_energy, check_per_atom, gpu_eval, note, rms_rel, soa_to_aos,
                        to_dev)
from paper_1809_07726_amd import synth

pytestmark = pytest.mark.gpu


def _sample_check(b, g, reps):
    off = b["atom_off"]
    for r in reps:
        a, c = off[r], off[r + 1]
        Eo, gx, _, _ = oracle.gradient(b["xyz"][a:c], b["q"][a:c], b["rho"][a:c], b["screen"][a:c],
                                       b["sigma"][a:c], b["eps"][a:c])
        check_energy(g["E"][r], Eo)
        check_per_atom(g["F"][a:c], -gx)


def _any_size_properties(b, g):
    off = b["atom_off"]
    assert np.all(np.isfinite(g["E"]))
    for r in range(off.size - 1):
        F = g["F"][off[r]:off[r + 1]]
        assert np.abs(F.sum(0)).max() <= 2e-8 * np.abs(F).sum() + 1e-9


def test_autograd_matches_oracle_gradient():
    """Two 4,096-atom replicas with independent jitter (the differentiation
    workload's shape); upstream gradient differs per replica."""
    from paper_1809_07726_amd.gb import Context, gb_energy
    b = synth.make_config(3, n_rep=2)
    d = to_dev(b)
    t = d.t
    ctx = Context(b["atom_off"])
    x = t["xyz"].clone().requires_grad_(True)
    q = t["q"].clone().requires_grad_(True)
    rho = t["rho"].clone().requires_grad_(True)
    E = gb_energy(x, q, rho, t["screen"], t["sigma"], t["eps"], ctx)
    w = torch.tensor([0.7, -1.3], dtype=torch.float64, device="cuda")
    (E * w).sum().backward()
    ctx.check()
    N = ctx.n_atoms
    gx = soa_to_aos(x.grad.cpu().numpy(), N)
    gq = q.grad.cpu().double().numpy()
    gr = rho.grad.cpu().double().numpy()
    Eg = E.detach().cpu().numpy()
    off = b["atom_off"]
    wn = w.cpu().numpy()
    for r in range(2):
        a, c = off[r], off[r + 1]
        Eo, ox, oq, orr = oracle.gradient(b["xyz"][a:c], b["q"][a:c], b["rho"][a:c], b["screen"][a:c],
                                          b["sigma"][a:c], b["eps"][a:c])
        rel = abs(Eg[r] - Eo.sum()) / abs(Eo.sum())
        note("energy rel", rel)
        assert rel <= 1e-6
        check_per_atom(gx[a:c], wn[r] * ox, "dE/dx")
        check_per_atom(gq[a:c], wn[r] * oq, "dE/dq")
        check_per_atom(gr[a:c], wn[r] * orr, "dE/drho")
    ctx.close()


def test_autograd_rejects_non_differentiable_inputs():
    from paper_1809_07726_amd.gb import Context, gb_energy
    b = synth.make_config(0, n_atoms=64)
    d = to_dev(b)
    t = d.t
    ctx = Context(b["atom_off"])
    scr = t["screen"].clone().requires_grad_(True)
    with pytest.raises(ValueError):
        gb_energy(t["xyz"], t["q"], t["rho"], scr, t["sigma"], t["eps"], ctx)
    ctx.close()


def test_uneven_batch_reduced():
    """The uneven workload's structure (log-uniform sizes, sites every ~200
    atoms, 4 pH replicas per system) at sizes the oracle finishes quickly."""
    b = synth.make_config(4, n_systems=6, n_atoms=2500)
    g = gpu_eval(b)
    _sample_check(b, g, range(b["n_rep"]))


def test_full_size_e_ph_t_batch_sampled():
    """192 x 1,024 (the benchmarked batch) in one launch per pass; three
    replicas checked element by element against the oracle."""
    b = synth.make_config(2, per_replica_jitter=True)
    g = gpu_eval(b)
    _sample_check(b, g, [0, 95, 191])
    _any_size_properties(b, g)


def test_full_size_e_ph_t_batch_in_the_tuned_launch():
    """The benchmarked batch in the launch configuration bench.py times: the
    autotuner's choice of register blocking and launch shape."""
    from paper_1809_07726_amd.gb import Context
    from paper_1809_07726_amd.tune import autotune
    b = synth.make_config(2, per_replica_jitter=True)
    ctx = Context(b["atom_off"])
    tuned = autotune(ctx, to_dev(b).t, reps=3)
    ctx.close()
    print("tuned launch:", tuned["shape"], tuned["blocking"], flush=True)
    g = gpu_eval(b, blocking=tuple(tuned["blocking"]), launch=tuple(tuned["shape"]))
    _sample_check(b, g, [7, 130])
    _any_size_properties(b, g)


def test_full_size_e_ph_batch_sampled():
    b = synth.make_config(1, per_replica_jitter=True)
    g = gpu_eval(b)
    _sample_check(b, g, [0, 47])
    _any_size_properties(b, g)


def test_full_size_gradient_batch_sampled():
    b = synth.make_config(3)
    g = gpu_eval(b)
    _sample_check(b, g, [5, 12])
    _any_size_properties(b, g)


def test_full_size_uneven_batch_sampled_and_deterministic():
    """64 systems of 500..20,000 atoms x 4 replicas: a replica of the smallest
    and of the largest system (19,762 atoms) against the oracle; all replicas
    finite, force-balanced and identical on a second run."""
    b = synth.make_config(4)
    g1 = gpu_eval(b)
    sizes = np.diff(b["atom_off"])
    r_small, r_large = int(np.argmin(sizes)), int(np.argmax(sizes))
    print(f"oracle on replicas of {sizes[r_small]} and {sizes[r_large]} atoms", flush=True)
    _sample_check(b, g1, [r_small, r_large])
    _any_size_properties(b, g1)
    g2 = gpu_eval(b)
    assert np.array_equal(g1["F_fx"], g2["F_fx"]) and np.array_equal(g1["E_fx"], g2["E_fx"])
    # replicas of one system share coordinates: identical energies across its 4 replicas
    E = g1["E"][:, 4].reshape(-1, 4)
    assert np.all(E == E[:, :1])


def test_blocked_20k_system_with_salt_and_packed_cutoff_lists_matches_oracle():
    """One 20,000-atom system in compact 64-atom blocks with salt and both
    cutoffs, so that the pair passes run packed work lists: energies, Born
    radii and forces against the oracle.  The atoms sit exactly on the 3.0 A
    lattice (no jitter), so every pair distance squared is a multiple of 9 A^2
    and cut = 12.1 A, rgbmax = 15.1 A lie far from any of them (no pair sits
    within FP32 rounding of a cutoff)."""
    import paper_1809_07726_amd._capi as A
    b = synth.make_config(5, n_atoms=20000)
    b["xyz"] = b["x0"].copy()
    P = A.obc2(kappa=0.1, cut=12.1, rgbmax=15.1)
    G = oracle.obc2(kappa=0.1, cut=12.1, rgbmax=15.1)
    g = gpu_eval(b, params=P)
    n = 20000
    Eo, gx, _, _ = oracle.gradient(b["xyz"], b["q"], b["rho"], b["screen"], b["sigma"], b["eps"], G)
    _, Ro, _ = oracle.born(b["xyz"], b["rho"], b["screen"], G)
    assert np.abs(g["R"] / Ro - 1).max() < 2e-6
    check_energy(g["E"][0], Eo)
    check_per_atom(g["F"], -gx)
    _any_size_properties(b, g)
    assert n == b["atom_off"][-1]


def test_full_size_100k_salt_cutoff_system_in_the_tuned_launch_sampled():
    """The 100,000-atom salt-and-cutoff system at its full size, in the
    launch the benchmark times (4 wavefronts x 8 workgroups per CU, one i
    atom per lane in every pass, packed lists), with the atoms exactly on the
    lattice (cut = 12.1 A, rgbmax = 15.1 A clear of every pair distance).
    Sampled against the oracle on exact subsystems (the locality of the cut-off
    sums is pinned on the CPU): the Born radii of 256 atoms (the atoms within
    rgbmax + 1 A) and the forces on 24 atoms (within cut + 2 rgbmax + 1 A)."""
    import paper_1809_07726_amd._capi as A
    b = synth.make_config(5)
    b["xyz"] = b["x0"].copy()
    cut, rgb = 12.1, 15.1
    P = A.obc2(kappa=0.1, cut=cut, rgbmax=rgb)
    G = oracle.obc2(kappa=0.1, cut=cut, rgbmax=rgb)
    print("case: 1 x 100,000 atoms, blocking (1, 1, 1), launch (4, 8)", flush=True)
    g = gpu_eval(b, params=P, blocking=(1, 1, 1), launch=(4, 8))
    _any_size_properties(b, g)
    x = b["xyz"].astype(np.float64)
    rng = np.random.default_rng(100)
    for i in rng.choice(len(x), 256, replace=False):
        near = np.flatnonzero(((x - x[i]) ** 2).sum(1) < (rgb + 1.0) ** 2)
        _, Rs, _ = oracle.born(x[near], b["rho"][near], b["screen"][near], G)
        assert abs(g["R"][i] / Rs[int(np.searchsorted(near, i))] - 1) < 2e-6, i
    F_rms = np.sqrt((g["F"] ** 2).sum(1).mean())
    for i in rng.choice(len(x), 24, replace=False):
        sel = np.flatnonzero(((x - x[i]) ** 2).sum(1) < (cut + 2 * rgb + 1.0) ** 2)
        _, gs, _, _ = oracle.gradient(x[sel], b["q"][sel], b["rho"][sel], b["screen"][sel], b["sigma"][sel],
                                      b["eps"][sel], G)
        Fo = -gs[int(np.searchsorted(sel, i))]
        assert np.linalg.norm(g["F"][i] - Fo) <= 1e-5 * max(np.linalg.norm(Fo), F_rms), (i, g["F"][i], Fo)


def test_repeated_evaluations_on_one_context_match_a_fresh_context():
    """The energy pass adds its sums into per-replica stripes that the next
    kernel folds into the energies and clears, and the packing rebuilds the
    cutoff lists at every evaluation: three evaluations in a row on one
    context give the bits of a fresh context, for the 192 x 1,024 batch
    (all-pairs lists) and for one 20,000-atom replica with packed lists (a
    stale stripe would double an energy)."""
    import paper_1809_07726_amd._capi as A
    from paper_1809_07726_amd.gb import Context
    b5 = synth.make_config(5, n_atoms=20000)
    b5["xyz"] = b5["x0"].copy()
    cases = [(b5, A.obc2(kappa=0.1, cut=12.1, rgbmax=15.1)), (synth.make_config(2), None)]
    for b, P in cases:
        ref = gpu_eval(b, params=P)
        ctx = Context(b["atom_off"], P)
        t = to_dev(b).t
        for k in range(3):
            R, dR, psi = ctx.born_radii(t["xyz"], t["rho"], t["screen"])
            f, e, _, _ = ctx.energy_forces(t["xyz"], t["q"], t["rho"], t["screen"], t["sigma"], t["eps"],
                                           R, dR, psi)
            ctx.check()
            e, f = e.cpu().numpy(), f.cpu().numpy()
            assert np.array_equal(e, ref["E_fx"]), (b["n_rep"], k)
            assert np.array_equal(f, ref["F_fx"]), (b["n_rep"], k)
        ctx.close()


def _jittered_20k():
    """20,000 atoms in compact 64-atom blocks with their lattice jitter (so
    pair distances are continuous and each I block's atoms come from up to
    five windows of the packing)."""
    return synth.make_config(5, n_atoms=20000)


def test_packed_lists_are_bit_reproducible_on_a_jittered_20k_system():
    """With salt and both cutoffs the packing places every J atom by the
    coordinates alone: two fresh contexts, in each of two blockings, give
    identical bits for radii, forces and energies."""
    import paper_1809_07726_amd._capi as A
    b = _jittered_20k()
    P = A.obc2(kappa=0.1, cut=12.0, rgbmax=15.0)
    for blk in ((1, 1, 1), (2, 2, 2)):
        print(f"case: jittered 20,000 atoms, blocking {blk}", flush=True)
        g1 = gpu_eval(b, True, True, blocking=blk, params=P)
        g2 = gpu_eval(b, True, True, blocking=blk, params=P)
        for k in ("R", "F_fx", "E_fx", "dEdq", "dEdrho"):
            assert np.array_equal(g1[k], g2[k]), (blk, k)


def test_jittered_20k_system_at_the_requested_cutoffs_matches_oracle():
    """Off the lattice and at the requested cutoffs (cut 12 A, rgbmax 15 A, no
    clearing): a pair whose distance lies within FP32 rounding of a cutoff may
    be counted on one side and not on the other.  FP64 lists the pairs within
    2e-5 A of either cutoff (about a hundred times the FP32 rounding of r):
      - Born radii: atoms in no such rgbmax pair within 2e-6 of the oracle; the
        others between the oracle's radii with rgbmax -+ 2e-5 A;
      - energies at the GPU's own radii (so that only the pair cutoff is left):
        within 1e-6 relative plus the summed |GB + C + LJ| pair energies of the
        pairs near cut (each from the oracle on the two atoms alone);
      - forces: 1e-5 RMS-relative against the oracle."""
    import paper_1809_07726_amd._capi as A
    from scipy.spatial import cKDTree
    b = _jittered_20k()
    cut, rgb, kap, dl = 12.0, 15.0, 0.1, 2e-5
    P = A.obc2(kappa=kap, cut=cut, rgbmax=rgb)
    G = oracle.obc2(kappa=kap, cut=cut, rgbmax=rgb)
    print("case: jittered 20,000 atoms, requested cutoffs", flush=True)
    g = gpu_eval(b, params=P)
    x = b["xyz"].astype(np.float64)
    tree = cKDTree(x)
    def near(rc):
        pr = tree.query_pairs(rc + dl, output_type="ndarray").astype(np.int64).reshape(-1, 2)
        r = np.sqrt(((x[pr[:, 0]] - x[pr[:, 1]]) ** 2).sum(1))
        return pr[np.abs(r - rc) < dl]
    near_cut, near_rgb = near(cut), near(rgb)
    print(f"pairs within {dl} A: {len(near_cut)} of cut, {len(near_rgb)} of rgbmax", flush=True)
    # Born radii
    _, Ro, _ = oracle.born(x, b["rho"], b["screen"], G)
    _, Rlo, _ = oracle.born(x, b["rho"], b["screen"], oracle.obc2(kappa=kap, cut=cut, rgbmax=rgb - dl))
    _, Rhi, _ = oracle.born(x, b["rho"], b["screen"], oracle.obc2(kappa=kap, cut=cut, rgbmax=rgb + dl))
    edge = np.zeros(len(x), bool)
    edge[near_rgb.reshape(-1)] = True
    rel = np.abs(g["R"] / Ro - 1)
    note("Born radius rel (off the rgbmax edge)", rel[~edge].max())
    assert rel[~edge].max() < 2e-6
    lo, hi = np.minimum(Rlo, Rhi), np.maximum(Rlo, Rhi)
    assert np.all(g["R"][edge] >= lo[edge] * (1 - 2e-6)) and np.all(g["R"][edge] <= hi[edge] * (1 + 2e-6))
    # energies at the GPU's radii
    Rg = g["R"].astype(np.float64)
    Eo = oracle.energy_at_R(x, b["q"], Rg, b["sigma"], b["eps"], G)
    free = oracle.obc2(kappa=kap)
    bound = 0.0
    for i, j in near_cut:
        two = oracle.energy_at_R(x[[i, j]], b["q"][[i, j]], Rg[[i, j]], b["sigma"][[i, j]], b["eps"][[i, j]], free)
        one = sum(oracle.energy_at_R(x[[k]], b["q"][[k]], Rg[[k]], b["sigma"][[k]], b["eps"][[k]], free)
                  for k in (i, j))
        bound += np.abs(two - one).sum()
    Eg = g["E"][0]
    err = abs(Eg[4] - Eo.sum())
    note("energy err over (1e-6 |E| + near-cut pair terms)", err / (1e-6 * abs(Eo.sum()) + bound))
    assert err <= 1e-6 * abs(Eo.sum()) + bound, (Eg, Eo, bound)
    assert abs(Eg[0] - Eo[0]) <= 1e-6 * abs(Eo[0]) + bound
    # forces
    _, gx, _, _ = oracle.gradient(x, b["q"], b["rho"], b["screen"], b["sigma"], b["eps"], G)
    e_rms = rms_rel(g["F"], -gx)
    note("force rms-rel", e_rms)
    assert e_rms < 1e-5
