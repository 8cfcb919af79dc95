"""md_step, titration Monte Carlo and replica exchange on the GPU against the
oracle: short trajectories (positions, velocities, charges, states,
energies), exchange decisions on identical inputs, graph replay equal to
eager launches, and titration statistics (eq. 1, eq. 2)."""
import math

import numpy as np
import pytest
import torch

import oracle
from common import (batch_mean_bound, diprotic_site_batch, three_state_expected, with_diprotic_ph_sites,
                    with_oracle_gref)
from gpu_common import FX_E, FX_F, soa_to_aos
from paper_1809_07726_amd import synth

pytestmark = pytest.mark.gpu


def _gpu_md(b, seed, steps_chunks, graph=False, init=True, params=None):
    from paper_1809_07726_amd.gb import MD, Context, DeviceBatch
    ctx = Context(b["atom_off"], params)
    d = DeviceBatch.from_numpy(b)
    md = MD(ctx, d, b, seed=seed)
    snaps = []
    first = True
    for n in steps_chunks:
        md.run(n, init_forces=init and first, graph=graph)
        first = False
        torch.cuda.synchronize()
        N = ctx.n_atoms
        snaps.append({
            "xyz": soa_to_aos(d.t["xyz"].cpu().numpy(), N), "v": soa_to_aos(d.t["v"].cpu().numpy(), N),
            "q": d.t["q"].cpu().numpy().astype(np.float64),
            "site_state": d.t["site_state"].cpu().numpy().copy() if b["n_sites"] else None,
            "target_idx": d.t["target_idx"].cpu().numpy().reshape(-1, 4).copy(),
            "grid_rep": d.t["grid_rep"].cpu().numpy().copy(),
            "E": md.energy_fx.cpu().numpy().reshape(-1, 4) * FX_E,
            "F_fx": md.force_fx.cpu().numpy().copy(),
            "ke": md.ke.cpu().numpy().copy(),
            "mc_stats": md.mc_stats.cpu().numpy().copy() if md.mc_stats is not None else None,
        })
    ctx.check()
    ctx.close()
    return snaps


def _oracle_md(b, seed, steps_chunks, gb=None):
    cfg, st, arr, keep = oracle.make_md(b, gb=gb, seed=seed)
    oracle.md_run(cfg, st, 0, 0, True)
    snaps, step = [], 0
    for n in steps_chunks:
        oracle.md_run(cfg, st, step, n, False)
        step += n
        snaps.append({k: arr[k].copy() for k in ("xyz", "v", "q", "site_state", "target_idx",
                                                 "grid_rep", "E", "F", "mc_att", "mc_acc",
                                                 "ex_att", "ex_acc")})
    return snaps


def test_md_step_matches_oracle_trajectory():
    """c0 system: 25 Langevin steps with titration attempts every 10 steps."""
    b = with_oracle_gref(synth.make_config(0))
    seed = 2000
    g = _gpu_md(b, seed, [10, 15])
    o = _oracle_md(b, seed, [10, 15])
    for gs, os_ in zip(g, o):
        x_o = os_["xyz"].reshape(-1, 3)
        v_o = os_["v"].reshape(-1, 3)
        assert np.abs(gs["xyz"] - x_o).max() < 2e-4
        assert np.sqrt(((gs["v"] - v_o) ** 2).sum() / (v_o ** 2).sum()) < 1e-3
        assert np.array_equal(gs["site_state"], os_["site_state"])
        assert np.allclose(gs["q"], os_["q"], atol=1e-6)
        Eo = os_["E"].reshape(-1, 4)
        assert np.allclose(gs["E"], Eo, rtol=1e-4, atol=1e-3)
    # the attempts counted on both sides
    assert g[-1]["mc_stats"][0::2].sum() == o[-1]["mc_att"].sum() == 4


def test_md_step_titration_on_a_replica_of_several_chunks_matches_oracle():
    """A 2,500-atom replica (its titration sums span two chunks of atoms):
    attempts every step for 6 steps follow the oracle's states exactly.  G_ref
    is the sites' energy change in the whole system at the start, so that the
    attempts are accepted about half of the time."""
    b = synth.make_config(0, n_atoms=2500, seed=1010)
    b["mc_every"] = 1
    _, R, _ = oracle.born(b["xyz"], b["rho"], b["screen"])
    ms = b["max_states"]
    for s in range(b["n_sites"]):
        sl = slice(b["site_off"][s], b["site_off"][s + 1])
        qn = b["state_q"].reshape(-1, ms)[sl, 1]
        b["G_ref"][s * ms + 1] = oracle.delta_e(b["xyz"], b["q"], R, b["site_atoms"][sl], qn)
    g = _gpu_md(b, 2300, [3, 3])
    o = _oracle_md(b, 2300, [3, 3])
    for gs, os_ in zip(g, o):
        assert np.array_equal(gs["site_state"], os_["site_state"])
        assert np.allclose(gs["q"], os_["q"], atol=1e-6)
        assert np.abs(gs["xyz"] - os_["xyz"].reshape(-1, 3)).max() < 1e-4
    assert g[-1]["mc_stats"][0::2].sum() == o[-1]["mc_att"].sum() == 12
    assert o[-1]["mc_acc"].sum() > 0


def test_md_first_step_is_exact_to_fp32():
    """One step from rest: the Ornstein-Uhlenbeck noise is the same Philox
    stream on both sides, so positions agree to FP32 rounding."""
    b = with_oracle_gref(synth.make_config(0))
    g = _gpu_md(b, 77, [1])[0]
    o = _oracle_md(b, 77, [1])[0]
    assert np.abs(g["xyz"] - o["xyz"].reshape(-1, 3)).max() < 1e-5
    v_o = o["v"].reshape(-1, 3)
    assert np.abs(g["v"] - v_o).max() < 1e-4 * np.abs(v_o).max()


def test_graph_replay_is_bitwise_equal_to_eager():
    b = with_oracle_gref(synth.make_config(1, n_atoms=256, n_rep=8))
    b["ex_every"] = 10
    eager = _gpu_md(b, 5, [35])[0]
    graph = _gpu_md(b, 5, [35], graph=True)[0]
    for k in ("xyz", "v", "q", "site_state", "target_idx", "grid_rep", "F_fx"):
        assert np.array_equal(eager[k], graph[k]), k


def test_graph_replay_with_hamiltonian_exchanges_is_bitwise_equal_to_eager():
    """Captured step graphs on a 2 T x 3 H grid (exchanges every 5 steps, so
    the graphs hold the Hamiltonian swaps and the force rescaling after
    them) give the same bits as eager launches."""
    base = synth.draw_system(160, 4343, 2, 1)
    reps = [synth.jitter_copy(base, 700 + r) for r in range(12)]
    b = synth.assemble([base, base], 6, (-0.2,), (7.0,), (300.0, 330.0), (synth.DIM_H, synth.DIM_T),
                       per_replica=reps, H_scale=(1.0, 0.9, 0.8), mc_every=5, ex_every=5)
    b = with_oracle_gref(b)
    eager = _gpu_md(b, 9, [12, 13])
    graph = _gpu_md(b, 9, [12, 13], graph=True)
    for e, g in zip(eager, graph):
        for k in ("xyz", "v", "q", "site_state", "target_idx", "grid_rep", "F_fx"):
            assert np.array_equal(e[k], g[k]), k
    assert not np.array_equal(eager[-1]["target_idx"][:, synth.DIM_H], b["target_idx"][:, synth.DIM_H])


def test_graph_replay_with_packed_cutoff_lists_is_bitwise_equal_to_eager():
    """Captured step graphs with salt and both cutoffs (the packing kernels and
    their counter resets inside the graphs, replayed many times, MC every 5
    steps and exchanges every 10) give the same bits as eager launches."""
    import paper_1809_07726_amd._capi as A
    from gpu_common import clear_cutoffs
    b = with_oracle_gref(synth.make_config(1, n_atoms=700, n_rep=4))
    b["mc_every"], b["ex_every"] = 5, 10
    cut, rgb = clear_cutoffs(b, 8.0, 10.0)
    P = A.obc2(kappa=0.1, cut=cut, rgbmax=rgb)
    eager = _gpu_md(b, 13, [12, 18], params=P)
    graph = _gpu_md(b, 13, [12, 18], graph=True, params=P)
    for e, g in zip(eager, graph):
        for k in ("xyz", "v", "q", "site_state", "target_idx", "grid_rep", "F_fx"):
            assert np.array_equal(e[k], g[k]), k


def test_gpu_hamiltonian_exchange_samples_the_pair_boltzmann_weights():
    """32 frozen two-replica systems on a 2-level Hamiltonian grid (scales 1.0
    and 0.8), exchange attempts every step on the GPU: each pair holds the
    arrangement (replica 0 at level 0) with probability w_A / (w_A + w_B) of
    the Boltzmann weights of the two arrangements, from the oracle's
    energies."""
    from paper_1809_07726_amd.gb import MD, Context, DeviceBatch
    lams = (1.0, 0.8)
    base = synth.draw_system(16, 51, 0, 0)
    base["sites"] = []
    pair = [synth.jitter_copy(base, s) for s in (3, 4)]
    b = synth.assemble([base] * 32, 2, (-0.2,), (7.0,), (300.0,), (synth.DIM_H,), per_replica=pair * 32,
                       H_scale=lams, dt=0.0, mc_every=0, ex_every=1)
    off = b["atom_off"]
    E = [oracle.energy(b["xyz"][off[r]:off[r + 1]], b["q"][off[r]:off[r + 1]], b["rho"][off[r]:off[r + 1]],
                       b["screen"][off[r]:off[r + 1]], b["sigma"][off[r]:off[r + 1]], b["eps"][off[r]:off[r + 1]]).sum()
         for r in (0, 1)]
    t = [oracle.tether(b["xyz"][off[r]:off[r + 1]], b["x0"][off[r]:off[r + 1]], b["k_tether"])[0] for r in (0, 1)]
    U = lambda r, lam: lam * E[r] + t[r]
    beta = 1.0 / (oracle.constants()["kB"] * 300.0)
    eA, eB = -beta * (U(0, lams[0]) + U(1, lams[1])), -beta * (U(0, lams[1]) + U(1, lams[0]))
    pA = 1.0 / (1.0 + math.exp(eB - eA))
    ctx = Context(off)
    d = DeviceBatch.from_numpy(b)
    md = MD(ctx, d, b, seed=77)
    md.run(1, init_forces=True)
    n = 400
    held = np.zeros((n, 32))
    for k in range(n):
        md.run(1)
        held[k] = d.t["target_idx"].cpu().numpy().reshape(-1, 4)[0::2, synth.DIM_H] == 0
    ctx.check()
    ctx.close()
    per_pair = held.mean(0)                     # 32 independent chains
    assert abs(per_pair.mean() - pA) <= batch_mean_bound(per_pair, 16), (per_pair.mean(), pA)


def test_exchange_inputs_on_a_hamiltonian_grid():
    """gbr_exchange_inputs on a 2 T x 3 H grid: enb is the unscaled
    E_GB + E_C + E_LJ of each replica and the temperature-exchange energy is
    that of the replica's own Hamiltonian, l (E_GB + E_C + E_LJ) + E_tether
    (eps_mode 1), both as the oracle forms them from the same energies."""
    from paper_1809_07726_amd.gb import MD, Context, DeviceBatch
    base = synth.draw_system(96, 4545, 1, 1)
    reps = [synth.jitter_copy(base, 800 + r) for r in range(6)]
    lams = (1.0, 0.85, 0.7)
    b = synth.assemble([base], 6, (-0.2,), (7.0,), (300.0, 330.0), (synth.DIM_H, synth.DIM_T),
                       per_replica=reps, H_scale=lams, mc_every=0, ex_every=0)
    ctx = Context(b["atom_off"])
    d = DeviceBatch.from_numpy(b)
    md = MD(ctx, d, b, seed=3, eps_mode=1)
    md.run(3, init_forces=True)
    nH, ne, eps, enb = (t.cpu().numpy() for t in md.exchange_inputs())
    E = md.energy_fx.cpu().numpy().reshape(-1, 4) * FX_E
    ti = d.t["target_idx"].cpu().numpy().reshape(-1, 4)
    ctx.check()
    ctx.close()
    W = E[:, :3].sum(1)
    lam = np.asarray(lams)[ti[:, synth.DIM_H]]
    assert np.allclose(enb, W, rtol=0, atol=1e-9 * np.abs(W).max())
    assert np.allclose(eps, lam * W + E[:, 3], rtol=0, atol=1e-9 * np.abs(W).max())
    cfg, st, arr, keep = oracle.make_md(b, seed=3, eps_mode=1)
    _, _, ep_o = oracle.replica_counts(cfg, b["site_state"], ti, E)
    assert np.allclose(eps, ep_o, rtol=0, atol=1e-9 * np.abs(W).max())


def test_replica_grid_md_with_exchanges_matches_oracle():
    """A 2 x 2 x 2 (E, T, pH) grid, 2 instances, MC every 5 steps and
    exchanges every 10: targets and states follow the oracle exactly."""
    base = synth.draw_system(160, 4242, 2, 1)
    b = synth.assemble([base, synth.jitter_copy(base, 99)], 8, (-0.25, -0.15), (6.0, 7.5),
                       (300.0, 330.0), (synth.DIM_E, synth.DIM_T, synth.DIM_PH),
                       mc_every=5, ex_every=10)
    b = with_oracle_gref(b)
    chunks = [10, 10, 10, 10]
    g = _gpu_md(b, 31, chunks)
    o = _oracle_md(b, 31, chunks)
    for gs, os_ in zip(g, o):
        assert np.array_equal(gs["target_idx"], os_["target_idx"].reshape(-1, 4))
        assert np.array_equal(gs["grid_rep"], os_["grid_rep"])
        assert np.array_equal(gs["site_state"], os_["site_state"])
        assert np.abs(gs["xyz"] - os_["xyz"].reshape(-1, 3)).max() < 1e-3


def test_hamiltonian_grid_md_matches_oracle():
    """A 2 T x 3 H grid (Hamiltonian scales 1.0, 0.9, 0.8 of the GB + Coulomb
    + LJ energy), 2 instances, MC and exchanges every 5 steps, T and H
    attempts alternating: targets, states and positions follow the oracle,
    and the forces at the end of each call (an exchange step, so the replicas
    that changed level hold forces rescaled to the new level) match its fresh
    evaluation."""
    base = synth.draw_system(160, 4343, 2, 1)
    reps = [synth.jitter_copy(base, 500 + r) for r in range(12)]
    b = synth.assemble([base, base], 6, (-0.2,), (7.0,), (300.0, 330.0), (synth.DIM_T, synth.DIM_H),
                       per_replica=reps, H_scale=(1.0, 0.9, 0.8), mc_every=5, ex_every=5)
    b = with_oracle_gref(b)
    chunks = [10, 10, 10, 10]
    g = _gpu_md(b, 41, chunks)
    o = _oracle_md(b, 41, chunks)
    N = b["atom_off"][-1]
    for gs, os_ in zip(g, o):
        assert np.array_equal(gs["target_idx"], os_["target_idx"].reshape(-1, 4))
        assert np.array_equal(gs["grid_rep"], os_["grid_rep"])
        assert np.array_equal(gs["site_state"], os_["site_state"])
        assert np.abs(gs["xyz"] - os_["xyz"].reshape(-1, 3)).max() < 1e-3
        F_g = soa_to_aos(gs["F_fx"] * FX_F, N)
        F_o = os_["F"].reshape(-1, 3)
        assert np.sqrt(((F_g - F_o) ** 2).sum() / (F_o ** 2).sum()) < 1e-4
    G = 12
    acc_H = o[-1]["ex_acc"][synth.DIM_H * G:(synth.DIM_H + 1) * G].sum()
    assert acc_H > 0 and o[-1]["ex_att"][synth.DIM_H * G:(synth.DIM_H + 1) * G].sum() > acc_H


def test_exchange_decisions_match_oracle_on_identical_inputs():
    """192 replicas on the 8 x 6 x 4 grid; random proton / electron counts and
    energies; 12 consecutive attempts cycle E, T, pH with alternating parity."""
    from paper_1809_07726_amd.gb import Context, DeviceBatch
    w = synth.CONFIGS[2]
    base = synth.draw_system(16, 77, 0, 0)
    b = synth.assemble([base], 192, w.E_vals, w.pH_vals, w.T_vals, w.dim_order)
    cfg, st, arr, keep = oracle.make_md(b, seed=123)
    d = DeviceBatch.from_numpy(b)
    ctx = Context(b["atom_off"])
    rng = np.random.default_rng(8)
    R = b["n_rep"]
    ti_o, gr_o = b["target_idx"].copy(), b["grid_rep"].copy()
    ti_g = torch.as_tensor(ti_o.reshape(-1).copy(), device="cuda")
    gr_g = torch.as_tensor(gr_o.copy(), device="cuda")
    for a in range(12):
        nH = rng.integers(0, 6, R).astype(np.int32)
        ne = rng.integers(0, 2, R).astype(np.int32)
        ep = rng.normal(-5000.0, 3.0, R)
        ti_o, gr_o, vs_o, att, acc = oracle.exchange(cfg, a, nH, ne, ep, ti_o, gr_o)
        vs_g = ctx.remd_exchange(d.grid, a, torch.as_tensor(nH, device="cuda"),
                                 torch.as_tensor(ne, device="cuda"),
                                 torch.as_tensor(ep, device="cuda"), ti_g, gr_g, seed=123)
        torch.cuda.synchronize()
        assert np.array_equal(ti_g.cpu().numpy().reshape(-1, 4), ti_o), a
        assert np.array_equal(gr_g.cpu().numpy(), gr_o), a
        assert np.allclose(vs_g.cpu().numpy(), vs_o, rtol=1e-6)
        assert acc.sum() > 0
    ctx.check()
    ctx.close()


def test_exchange_decisions_with_a_hamiltonian_dimension_match_oracle():
    """2 instances of a 2 E x 2 pH x 2 T x 3 H grid; random counts and energy
    components (the GPU reads the unscaled E_GB + E_C + E_LJ, the oracle the
    four components); 16 attempts cycle E, H, T, pH."""
    from paper_1809_07726_amd.gb import Context, DeviceBatch
    base = synth.draw_system(16, 78, 0, 0)
    b = synth.assemble([base, base], 24, (-0.25, -0.2), (6.0, 7.0), (300.0, 320.0),
                       (synth.DIM_E, synth.DIM_H, synth.DIM_T, synth.DIM_PH), H_scale=(1.0, 0.95, 0.9))
    cfg, st, arr, keep = oracle.make_md(b, seed=321)
    d = DeviceBatch.from_numpy(b)
    ctx = Context(b["atom_off"])
    rng = np.random.default_rng(9)
    R = b["n_rep"]
    ti_o, gr_o = b["target_idx"].copy(), b["grid_rep"].copy()
    ti_g = torch.as_tensor(ti_o.reshape(-1).copy(), device="cuda")
    gr_g = torch.as_tensor(gr_o.copy(), device="cuda")
    n_acc_h = 0
    for a in range(16):
        nH = rng.integers(0, 6, R).astype(np.int32)
        ne = rng.integers(0, 2, R).astype(np.int32)
        ep = rng.normal(-5000.0, 3.0, R)
        E4 = np.stack([rng.normal(-300.0, 10.0, R), rng.normal(-50.0, 10.0, R),
                       rng.normal(-20.0, 5.0, R), rng.uniform(0.0, 5.0, R)], axis=1)
        ti_o, gr_o, vs_o, att, acc = oracle.exchange(cfg, a, nH, ne, ep, ti_o, gr_o, E4)
        vs_g = ctx.remd_exchange(d.grid, a, torch.as_tensor(nH, device="cuda"),
                                 torch.as_tensor(ne, device="cuda"),
                                 torch.as_tensor(ep, device="cuda"), ti_g, gr_g, seed=321,
                                 enb=torch.as_tensor(E4[:, :3].sum(1), device="cuda"))
        torch.cuda.synchronize()
        assert np.array_equal(ti_g.cpu().numpy().reshape(-1, 4), ti_o), a
        assert np.array_equal(gr_g.cpu().numpy(), gr_o), a
        assert np.allclose(vs_g.cpu().numpy(), vs_o, rtol=1e-6)
        n_acc_h += acc[synth.DIM_H * R:(synth.DIM_H + 1) * R].sum()
    assert n_acc_h > 0
    ctx.check()
    ctx.close()


@pytest.mark.parametrize("kind,delta", [("ph", -1.0), ("ph", 0.0), ("ph", 0.7),
                                        ("redox", -0.05), ("redox", 0.03)])
def test_gpu_titration_statistics(kind, delta):
    """Frozen isolated site, attempts every step on the GPU: the sampled
    fraction follows eq. 1 (pH) or eq. 2 (redox potential)."""
    from paper_1809_07726_amd.gb import reference_energies
    src = synth.make_config(0, n_atoms=64, seed=31)
    s = 0 if kind == "ph" else 1
    a, c = src["site_off"][s], src["site_off"][s + 1]
    idx = src["site_atoms"][a:c]
    t = synth.PH_SITE if kind == "ph" else synth.REDOX_SITE
    sysd = {k: src[k][idx] for k in ("xyz", "x0", "q", "rho", "screen", "sigma", "eps", "mass")}
    sysd["sites"] = [{"type": t, "atoms": np.arange(c - a), "q_states": src["state_q"].reshape(-1, 2)[a:c],
                      "nH": [0, 1] if t == 0 else [0, 0], "ne": [0, 0] if t == 0 else [0, 1],
                      "ref": src["ref_value"][s]}]
    # 64 independent copies of the site, each its own replica: more samples per step
    reps = 64
    E_vals = (synth.E0_REF + delta,) if kind == "redox" else (-0.2,)
    pH_vals = (synth.PKA_REF + delta,) if kind == "ph" else (7.0,)
    b = synth.assemble([sysd] * reps, 1, E_vals, pH_vals, (300.0,), (0,), dt=0.0, mc_every=1)
    b["G_ref"] = reference_energies(b)          # the HIP path's own reference compound
    from paper_1809_07726_amd.gb import MD, Context, DeviceBatch
    ctx = Context(b["atom_off"])
    d = DeviceBatch.from_numpy(b)
    md = MD(ctx, d, b, seed=900 + int(100 * delta))
    md.run(1, init_forces=True)
    n, occ = 400, 0.0
    for _ in range(n):
        md.run(1)
        occ += d.t["site_state"].float().mean().item()
    ctx.check()
    f_hat = occ / n
    if kind == "ph":
        f = 1.0 / (1.0 + 10.0 ** delta)
        up, down = min(1.0, 10.0 ** -delta), min(1.0, 10.0 ** delta)
    else:
        x = oracle.constants()["F"] * delta / (oracle.constants()["kB"] * 300.0)
        f = 1.0 / (1.0 + math.exp(x))
        up, down = min(1.0, math.exp(-x)), min(1.0, math.exp(x))
    lam = 1.0 - up - down
    sigma = math.sqrt(f * (1 - f) / (n * reps) * (1 + lam) / max(1 - lam, 1e-12))
    assert abs(f_hat - f) <= 4 * sigma + 1.0 / (n * reps), (f_hat, f, sigma)
    ctx.close()


def test_md_step_with_three_state_sites_matches_oracle():
    """c0 with its pH site given a third (doubly protonated) state and attempts
    every step: 25 steps follow the oracle's states exactly."""
    b = with_oracle_gref(with_diprotic_ph_sites(synth.make_config(0)))
    b["mc_every"] = 1
    seed = 2100
    g = _gpu_md(b, seed, [10, 15])
    o = _oracle_md(b, seed, [10, 15])
    for gs, os_ in zip(g, o):
        assert np.array_equal(gs["site_state"], os_["site_state"])
        assert np.allclose(gs["q"], os_["q"], atol=1e-6)
        assert np.abs(gs["xyz"] - os_["xyz"].reshape(-1, 3)).max() < 2e-4
    assert g[-1]["mc_stats"][0::2].sum() == o[-1]["mc_att"].sum() == 2 * 25


@pytest.mark.parametrize("d,tautomer", [(-0.5, False), (0.0, False), (0.5, False), (-0.5, True), (0.5, True)])
def test_gpu_three_state_site_statistics(d, tautomer):
    """64 frozen copies of an isolated three-state pH site (N_H = 0, 1, 2, or
    a deprotonated state and two protonated tautomers, N_H = 0, 1, 1),
    attempts every step on the GPU: the occupancies follow
    p(s) proportional to 10^(-(pH - pKa) N_H(s))."""
    from paper_1809_07726_amd.gb import MD, Context, DeviceBatch, reference_energies
    b = diprotic_site_batch(synth.PKA_REF + d, reps=64, tautomer=tautomer)
    b["G_ref"] = reference_energies(b)          # the HIP path's own reference compound
    ctx = Context(b["atom_off"])
    dv = DeviceBatch.from_numpy(b)
    md = MD(ctx, dv, b, seed=950 + int(100 * d) + 7 * tautomer)
    md.run(1, init_forces=True)
    n = 300
    occ = np.zeros((n, 64), np.int64)
    for k in range(n):
        md.run(1)
        occ[k] = dv.t["site_state"].cpu().numpy()
    ctx.check()
    ctx.close()
    p = three_state_expected(d, tautomer)
    for s in range(3):
        per_rep = (occ == s).mean(0)            # 64 independent chains
        assert abs(per_rep.mean() - p[s]) <= batch_mean_bound(per_rep, 16), (s, per_rep.mean(), p[s])


def test_md_step_with_salt_and_cutoffs_matches_oracle():
    """c0 with salt (kappa = 0.1 / A) and both cutoffs (near 9 and 11 A, clear of
    every starting pair distance): one step from rest to FP32 rounding.  Then
    25 steps with salt alone and titration attempts every 10 (with cutoffs, a
    pair that the trajectory carries across a cutoff within FP32 rounding of
    it may be counted at different steps on the two sides)."""
    import paper_1809_07726_amd._capi as A
    from gpu_common import clear_cutoffs
    base = synth.make_config(0)
    cut, rgb = clear_cutoffs(base, 9.0, 11.0)
    P = A.obc2(kappa=0.1, cut=cut, rgbmax=rgb)
    G = oracle.obc2(kappa=0.1, cut=cut, rgbmax=rgb)
    b = with_oracle_gref(base, G)
    g = _gpu_md(b, 78, [1], params=P)[0]
    o = _oracle_md(b, 78, [1], gb=G)[0]
    assert np.abs(g["xyz"] - o["xyz"].reshape(-1, 3)).max() < 1e-5
    v_o = o["v"].reshape(-1, 3)
    assert np.abs(g["v"] - v_o).max() < 1e-4 * np.abs(v_o).max()
    P, G = A.obc2(kappa=0.1), oracle.obc2(kappa=0.1)
    b = with_oracle_gref(base, G)
    seed = 2200
    g = _gpu_md(b, seed, [10, 15], params=P)
    o = _oracle_md(b, seed, [10, 15], gb=G)
    for gs, os_ in zip(g, o):
        assert np.abs(gs["xyz"] - os_["xyz"].reshape(-1, 3)).max() < 2e-4
        assert np.array_equal(gs["site_state"], os_["site_state"])
        Eo = os_["E"].reshape(-1, 4)
        assert np.allclose(gs["E"], Eo, rtol=1e-4, atol=1e-3)
