"""Multidimensional E,pH,T-REMD on the GPU, read through the analysis layer:
replica walks over the whole grid, exchange and MC acceptance against the
oracle's, and the eq. 1 / eq. 2 fits per grid point against eqs. 7-8 of a
frozen coupled pH + redox site, whose four state energies the oracle
enumerates exactly."""
import numpy as np
import pytest
import torch

import oracle
from common import coupled_sites_system, four_state_constants, four_state_energies
from gpu_common import note
from paper_1809_07726_amd import analysis as A

pytestmark = pytest.mark.gpu

TS = (300.0, 330.0)


def _grid():
    b0 = coupled_sites_system()
    eps = four_state_energies(b0)
    K = {T: four_state_constants(eps, T, b0["ref_value"][0], b0["ref_value"][1]) for T in TS}
    k = K[TS[0]]
    pHs = tuple(np.round(np.linspace(k["pKa_oxi"] - 1.5, k["pKa_red"] + 1.5, 5), 3))
    e_mid = float(A.eq7_e0(np.mean(pHs), k["E0_prot"], [k["pKa_red"]], [k["pKa_oxi"]], TS[0]))
    Es = tuple(np.round(np.linspace(e_mid - 0.08, e_mid + 0.08, 5), 4))
    return K, pHs, Es


def _rates(ex, mc_att, mc_acc, site_type, n_inst):
    r = A.exchange_acceptance(ex, n_inst, 5, 5, len(TS))
    out = {d: r[d]["rate"] for d in A.DIMS if r[d]["attempts"]}     # dimensions attempted
    for t, name in ((0, "mc_pH"), (1, "mc_redox")):
        m = site_type == t
        out[name] = mc_acc[m].sum() / mc_att[m].sum()
    return out


def test_e_ph_t_remd_walks_acceptance_and_titration_fits():
    from paper_1809_07726_amd.gb import MD, Context, DeviceBatch
    K, pHs, Es = _grid()
    n_inst, n_snap, every = 8, 4000, 2
    b = coupled_sites_system(pH_vals=pHs, E_vals=Es, T_vals=TS, n_inst=n_inst)
    ctx = Context(b["atom_off"])
    d = DeviceBatch.from_numpy(b)
    md = MD(ctx, d, b, seed=4321)
    md.run(0, init_forces=True)
    tg = torch.empty((n_snap,) + d.t["target_idx"].shape, dtype=d.t["target_idx"].dtype, device="cuda")
    ss = torch.empty((n_snap,) + d.t["site_state"].shape, dtype=d.t["site_state"].dtype, device="cuda")
    for i in range(n_snap):
        md.run(every)
        tg[i].copy_(d.t["target_idx"])
        ss[i].copy_(d.t["site_state"])
    torch.cuda.synchronize()
    ctx.check()
    tg = tg.cpu().numpy().reshape(n_snap, -1, 4)
    ss = ss.cpu().numpy()
    mc = md.mc_stats.cpu().numpy().astype(np.int64).reshape(-1, 2)
    g_rates = _rates(md.ex_stats.cpu().numpy(), mc[:, 0], mc[:, 1], b["site_type"], n_inst)
    ctx.close()

    # f1: every replica of every instance walks the whole 5 x 5 x 2 grid
    ws = A.walk_summary(A.residence_histogram(tg, 5, 5, len(TS)))
    note("residence max/min, worst replica", ws["worst_ratio"])
    note("residence max/min, median replica", np.median(ws["max_min_ratio"]))
    # 4,000 snapshots over 50 points: the worst of 400 replicas measured 3.8
    assert ws["fraction_visited_all"] == 1.0 and ws["worst_ratio"] < 5.0, ws["worst_ratio"]
    # every replica stays on a permutation of its instance's grid
    G = 5 * 5 * len(TS)
    gi = A.grid_index(tg, 5, len(TS)).reshape(n_snap, n_inst, G)
    assert np.all(np.sort(gi, axis=2) == np.arange(G))

    # acceptance per dimension and per site kind against the oracle on the same model
    bo = coupled_sites_system(pH_vals=pHs, E_vals=Es, T_vals=TS, n_inst=2)
    cfg, st, arr, keep = oracle.make_md(bo, seed=99)
    oracle.md_run(cfg, st, 0, 0, True)
    oracle.md_run(cfg, st, 0, 2000, False)
    o_rates = _rates(np.concatenate([arr["ex_att"], arr["ex_acc"]]), arr["mc_att"], arr["mc_acc"],
                     bo["site_type"], 2)
    assert set(g_rates) == set(o_rates) == {"E", "pH", "T", "mc_pH", "mc_redox"}
    for key in o_rates:
        assert abs(g_rates[key] - o_rates[key]) < 0.02, (key, g_rates[key], o_rates[key])

    # f2: E0 per (pH, T) against eq. 7 and pKa per (E, T) against eq. 8
    occ, n = A.fractions_per_point(ss, tg, b["rep_site_off"], 5, 5, len(TS))
    assert n.min() == n.max() == n_snap * n_inst
    fH = occ[:, 0].reshape(5, 5, len(TS))
    fR = occ[:, 1].reshape(5, 5, len(TS))
    for iT, T in enumerate(TS):
        k = K[T]
        for ip, pH in enumerate(pHs):
            e_fit, hill = A.fit_e0(Es, fR[:, ip, iT], T)
            e_pred = float(A.eq7_e0(pH, k["E0_prot"], [k["pKa_red"]], [k["pKa_oxi"]], T))
            assert abs(e_fit - e_pred) < 0.004 and abs(hill - 1) < 0.1, (T, pH, e_fit, e_pred, hill)
        for ie, E in enumerate(Es):
            p_fit, hill = A.fit_pka(pHs, fH[ie, :, iT])
            p_pred = float(A.eq8_sum_pka(E, k["E0_prot"], k["E0_deprot"], k["pKa_red"], T))
            assert abs(p_fit - p_pred) < 0.12 and abs(hill - 1) < 0.1, (T, E, p_fit, p_pred, hill)


def test_fig7_analogue_every_replica_visits_every_e_t_ph_combination():
    """The walk check of the paper's Fig. 7 on a grid of the 192-replica
    E,T,pH shape: 8 redox potentials 30 mV apart, 4 temperatures 20 K apart and
    6 pH values 0.5 apart (the paper's spacings), one instance of the frozen
    coupled-site model.  Every replica must visit all 192 combinations; the
    most to least visited ratio per replica and the acceptance per dimension
    are recorded, and the acceptances are held to the oracle's on the same
    grid."""
    from paper_1809_07726_amd.gb import MD, Context, DeviceBatch
    b0 = coupled_sites_system()
    k = four_state_constants(four_state_energies(b0), 300.0, b0["ref_value"][0], b0["ref_value"][1])
    pc = 0.5 * (k["pKa_oxi"] + k["pKa_red"])
    pHs = tuple(np.round(pc + 0.5 * (np.arange(6) - 2.5), 3))
    e_mid = float(A.eq7_e0(np.mean(pHs), k["E0_prot"], [k["pKa_red"]], [k["pKa_oxi"]], 300.0))
    Es = tuple(np.round(e_mid + 0.03 * (np.arange(8) - 3.5), 4))
    Ts = (280.0, 300.0, 320.0, 340.0)
    nE, npH, nT = len(Es), len(pHs), len(Ts)
    G = nE * npH * nT
    b = coupled_sites_system(pH_vals=pHs, E_vals=Es, T_vals=Ts, n_inst=1)
    ctx = Context(b["atom_off"])
    d = DeviceBatch.from_numpy(b)
    md = MD(ctx, d, b, seed=777)
    md.run(0, init_forces=True)
    n_chunks, chunk, every = 12, 4000, 2
    mult = torch.tensor([npH * nT, nT, 1, 0], dtype=torch.int64, device="cuda")
    rep = torch.arange(G, dtype=torch.int64, device="cuda") * G
    counts = torch.zeros(G * G, dtype=torch.int64, device="cuda")
    buf = torch.empty((chunk,) + d.t["target_idx"].shape, dtype=d.t["target_idx"].dtype, device="cuda")
    ratios = []
    for c in range(n_chunks):
        for i in range(chunk):
            md.run(every)
            buf[i].copy_(d.t["target_idx"])
        g = (buf.view(chunk, G, 4).long() * mult).sum(-1) + rep
        counts += torch.bincount(g.reshape(-1), minlength=G * G)
        ratios.append(A.walk_summary(counts.view(G, G).cpu().numpy())["worst_ratio"])
    torch.cuda.synchronize()
    ctx.check()
    ws = A.walk_summary(counts.view(G, G).cpu().numpy())
    r = A.exchange_acceptance(md.ex_stats.cpu().numpy(), 1, nE, npH, nT)
    ctx.close()
    for n, rt in zip((chunk * (c + 1) for c in range(n_chunks)), ratios):
        note(f"Fig. 7 grid: worst max/min after {n:>5} exchanges", rt)
    note("Fig. 7 grid: max/min, median replica", np.median(ws["max_min_ratio"]))
    for dim in ("E", "pH", "T"):
        note(f"Fig. 7 grid: {dim} acceptance", r[dim]["rate"])
    assert ws["fraction_visited_all"] == 1.0
    # the paper reports at most 2.2 for the replicas it shows; 48,000 attempts
    # bring every one of the 192 replicas below that (1.92 measured)
    assert ws["worst_ratio"] < 2.2, ws["worst_ratio"]

    bo = coupled_sites_system(pH_vals=pHs, E_vals=Es, T_vals=Ts, n_inst=1)
    cfg, st, arr, keep = oracle.make_md(bo, seed=99)
    oracle.md_run(cfg, st, 0, 0, True)
    oracle.md_run(cfg, st, 0, 1000, False)
    ro = A.exchange_acceptance(np.concatenate([arr["ex_att"], arr["ex_acc"]]), 1, nE, npH, nT)
    for dim in ("E", "pH", "T"):
        assert abs(r[dim]["rate"] - ro[dim]["rate"]) < 0.02, (dim, r[dim]["rate"], ro[dim]["rate"])
