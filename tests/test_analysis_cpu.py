"""The analysis layer (exchange diagnostics, eq. 1 / eq. 2 fits, eqs. 6-8)
pinned to exact data, to the 4-state enumeration of the oracle's frozen
coupled-site model, and end to end on an oracle E,pH-REMD run."""
import math

import numpy as np
import pytest

import oracle
from common import coupled_sites_system, four_state_constants, four_state_energies, four_state_probs
from paper_1809_07726_amd import analysis as A

C = oracle.constants()


def test_constants_agree_with_the_oracle():
    assert A.KB == C["kB"] and A.FARADAY == C["F"]
    assert A.LN10 == pytest.approx(C["ln10"], rel=1e-16)


@pytest.mark.parametrize("pka,n", [(4.85, 1.0), (6.2, 0.8), (7.1, 1.3)])
def test_fit_pka_recovers_eq1(pka, n):
    pH = np.linspace(pka - 2, pka + 2, 9)
    f = 1.0 / (1.0 + np.exp(n * math.log(10) * (pH - pka)))
    p, nn = A.fit_pka(pH, f)
    assert p == pytest.approx(pka, abs=1e-10) and nn == pytest.approx(n, rel=1e-10)


@pytest.mark.parametrize("e0,n,T", [(-0.203, 1.0, 300.0), (-0.15, 0.9, 340.0)])
def test_fit_e0_recovers_eq2(e0, n, T):
    E = np.linspace(e0 - 0.1, e0 + 0.1, 7)
    f = 1.0 / (1.0 + np.exp(n * C["F"] / (C["kB"] * T) * (E - e0)))
    e, nn = A.fit_e0(E, f, T)
    assert e == pytest.approx(e0, abs=1e-12) and nn == pytest.approx(n, rel=1e-10)


def test_eqs_6_7_8_against_enumeration_of_the_coupled_model():
    b = coupled_sites_system()
    eps = four_state_energies(b)
    T, pKa, E0 = 300.0, b["ref_value"][0], b["ref_value"][1]
    k = four_state_constants(eps, T, pKa, E0)
    # eq. 6
    assert k["E0_prot"] - k["E0_deprot"] == pytest.approx(
        A.eq6_shift([k["pKa_red"]], [k["pKa_oxi"]], T), rel=1e-10)
    from scipy.optimize import brentq
    for pH in np.linspace(3, 10, 8):
        e_enum = brentq(lambda E: four_state_probs(eps, pH, E, T, pKa, E0)[:, 1].sum() - 0.5, -2, 2,
                        xtol=1e-14)
        assert A.eq7_e0(pH, k["E0_prot"], [k["pKa_red"]], [k["pKa_oxi"]], T) == pytest.approx(e_enum, abs=1e-9)
    for E in np.linspace(-0.5, 0.1, 7):
        p_enum = brentq(lambda p: four_state_probs(eps, p, E, T, pKa, E0)[1, :].sum() - 0.5, -10, 25,
                        xtol=1e-13)
        assert A.eq8_sum_pka(E, k["E0_prot"], k["E0_deprot"], k["pKa_red"], T) == pytest.approx(p_enum, abs=1e-9)
    # limits stated with the equations: low pH -> E0_prot, high pH -> E0_deprot
    assert A.eq7_e0(-5.0, k["E0_prot"], [k["pKa_red"]], [k["pKa_oxi"]], T) == pytest.approx(k["E0_prot"], abs=1e-9)
    assert A.eq7_e0(20.0, k["E0_prot"], [k["pKa_red"]], [k["pKa_oxi"]], T) == pytest.approx(k["E0_deprot"], abs=1e-9)


def test_residence_histogram_and_acceptance_bookkeeping():
    # 2 x 1 x 2 x 1 grid (E, pH, T, H), 4 replicas; replica 0 walks 0 -> 1 -> 3 -> 3
    nE, npH, nT = 2, 1, 2
    snaps = np.array([
        [[0, 0, 0, 0], [0, 0, 1, 0], [1, 0, 0, 0], [1, 0, 1, 0]],
        [[0, 0, 1, 0], [0, 0, 0, 0], [1, 0, 0, 0], [1, 0, 1, 0]],
        [[1, 0, 1, 0], [0, 0, 0, 0], [1, 0, 0, 0], [0, 0, 1, 0]],
        [[1, 0, 1, 0], [0, 0, 0, 0], [1, 0, 0, 0], [0, 0, 1, 0]],
    ])
    h = A.residence_histogram(snaps, nE, npH, nT)
    assert h[0].tolist() == [1, 1, 0, 2]
    assert h.sum() == 16
    s = A.walk_summary(h)
    assert not s["visited_all"][0] and s["worst_ratio"] == math.inf
    ex = np.zeros(2 * 4 * 4, np.int64)
    ex[0 * 4 + 0] = 10; ex[16 + 0 * 4 + 0] = 4          # E attempts / accepts at point 0
    ex[2 * 4 + 1] = 5; ex[16 + 2 * 4 + 1] = 5           # T at point 1
    r = A.exchange_acceptance(ex, 1, nE, npH, nT)
    assert r["E"]["rate"] == 0.4 and r["T"]["rate"] == 1.0 and math.isnan(r["pH"]["rate"])
    assert math.isnan(r["H"]["rate"])
    # the same walk on a 1 x 1 x 2 x 2 grid (T, H): g = iT * nHam + iH
    snaps_h = snaps[..., [3, 1, 0, 2]]
    assert np.array_equal(A.residence_histogram(snaps_h, 1, 1, 2, 2), h)


def test_oracle_remd_walk_and_e0_fits_follow_eq7():
    """Frozen coupled pH + redox site on a 5 x 5 (E, pH) grid under the
    oracle's MC + exchange: every replica visits every grid point, E0 fitted
    per pH with eq. 2 follows eq. 7 of the model and pKa fitted per E with eq. 1
    follows eq. 8, within sampling error."""
    T = 300.0
    b0 = coupled_sites_system()
    eps = four_state_energies(b0)
    pKa, E0 = b0["ref_value"][0], b0["ref_value"][1]
    k = four_state_constants(eps, T, pKa, E0)
    pHs = tuple(np.round(np.linspace(k["pKa_oxi"] - 1.5, k["pKa_red"] + 1.5, 5), 3))
    e_mid = float(A.eq7_e0(np.mean(pHs), k["E0_prot"], [k["pKa_red"]], [k["pKa_oxi"]], T))
    Es = tuple(np.round(np.linspace(e_mid - 0.08, e_mid + 0.08, 5), 4))
    b = coupled_sites_system(pH_vals=pHs, E_vals=Es)
    cfg, st, arr, keep = oracle.make_md(b, seed=1234)
    oracle.md_run(cfg, st, 0, 0, True)
    states, targets = [], []
    step = 0
    for _ in range(1500):
        oracle.md_run(cfg, st, step, 4, False)
        step += 4
        states.append(arr["site_state"].copy())
        targets.append(arr["target_idx"].reshape(-1, 4).copy())
    h = A.residence_histogram(targets, len(Es), len(pHs), 1)
    assert A.walk_summary(h)["fraction_visited_all"] == 1.0
    occ, n = A.fractions_per_point(states, targets, b["rep_site_off"], len(Es), len(pHs), 1)
    f_red = occ[:, 1].reshape(len(Es), len(pHs))            # g = iE * npH + ipH
    for ip, pH in enumerate(pHs):
        e_fit, n_fit = A.fit_e0(Es, f_red[:, ip], T)
        e_pred = float(A.eq7_e0(pH, k["E0_prot"], [k["pKa_red"]], [k["pKa_oxi"]], T))
        assert abs(e_fit - e_pred) < 0.006, (pH, e_fit, e_pred)
    f_prot = occ[:, 0].reshape(len(Es), len(pHs))
    for ie, E in enumerate(Es):
        p_fit, n_fit = A.fit_pka(pHs, f_prot[ie])
        p_pred = float(A.eq8_sum_pka(E, k["E0_prot"], k["E0_deprot"], k["pKa_red"], T))
        assert abs(p_fit - p_pred) < 0.2, (E, p_fit, p_pred)
