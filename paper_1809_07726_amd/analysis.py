"""Analysis of multidimensional C(pH,E)MD / REMD runs.

Exchange diagnostics (what the paper reports about replica walks in its
Results, "Temperature dependence ..." subsection and Fig. 7): per-replica
residence histograms over the E x pH x T (x H) target grid and per-dimension
acceptance from the on-device counters of md_step.

Titration analysis (Theory, eqs. 1-2 and 6-8): protonated / reduced fractions
per grid point, fits of eq. 1 (pKa and Hill coefficient) and eq. 2 (E0 and
Hill coefficient), and the predictions of eqs. 6-8 from E0_prot, E0_deprot,
pKa_red and pKa_oxi.

Everything here is host-side numpy on data already produced by the device
(site states, target indices, counters); nothing in the hot path depends on it.
"""
from __future__ import annotations

import math

import numpy as np

KB = 0.001987204259        # kcal/(mol K), CODATA 2018 R / 4184
FARADAY = 23.0605480       # kcal/(mol V), CODATA 2018 F / 4184
LN10 = math.log(10.0)
DIMS = ("E", "pH", "T", "H")


# ------------------------------------------------------------------ grid
def grid_index(target_idx, npH: int, nT: int, nHam: int = 1):
    """Grid point g = ((iE * npH + ipH) * nT + iT) * nHam + iH for target rows
    [.., 4]."""
    t = np.asarray(target_idx)
    return ((t[..., 0] * npH + t[..., 1]) * nT + t[..., 2]) * nHam + t[..., 3]


def residence_histogram(target_snapshots, nE: int, npH: int, nT: int, nHam: int = 1):
    """counts[r, g]: number of snapshots in which replica r sat at grid point g
    (snapshots: [n_snap, n_rep, 4] target indices)."""
    s = np.asarray(target_snapshots)
    g = grid_index(s, npH, nT, nHam)               # [n_snap, n_rep]
    G = nE * npH * nT * nHam
    n_rep = s.shape[1]
    counts = np.zeros((n_rep, G), dtype=np.int64)
    for r in range(n_rep):
        counts[r] = np.bincount(g[:, r], minlength=G)
    return counts


def walk_summary(counts, n_inst: int = 1):
    """Per replica: whether it visited every point of its grid instance, and
    the ratio of its most to least visited point (inf if a point was missed)."""
    counts = np.asarray(counts)
    n_rep, G = counts.shape
    visited_all = (counts > 0).all(axis=1)
    ratio = np.where(visited_all, counts.max(axis=1) / np.maximum(counts.min(axis=1), 1), np.inf)
    return {"visited_all": visited_all, "max_min_ratio": ratio,
            "fraction_visited_all": float(visited_all.mean()),
            "worst_ratio": float(ratio.max())}


def exchange_acceptance(ex_stats, n_inst: int, nE: int, npH: int, nT: int, nHam: int = 1):
    """From md_step's ex_stats counters ([attempts(4 G_tot), accepts(4 G_tot)],
    indexed dim * G_tot + global lower grid point): acceptance per dimension and
    per lower grid point."""
    GT = n_inst * nE * npH * nT * nHam
    st = np.asarray(ex_stats, dtype=np.int64).reshape(2, len(DIMS), GT)
    att, acc = st[0], st[1]
    out = {}
    for d, name in enumerate(DIMS):
        a, c = att[d].sum(), acc[d].sum()
        out[name] = {"attempts": int(a), "accepts": int(c), "rate": float(c / a) if a else float("nan"),
                     "per_point": np.divide(acc[d], att[d], out=np.full(GT, np.nan), where=att[d] > 0)}
    return out


def mc_acceptance(mc_stats):
    st = np.asarray(mc_stats, dtype=np.int64).reshape(-1, 2)
    return {"attempts": st[:, 0], "accepts": st[:, 1],
            "rate": np.divide(st[:, 1], st[:, 0], out=np.full(len(st), np.nan), where=st[:, 0] > 0)}


# ------------------------------------------------------------ fractions
def fractions_per_point(state_snapshots, target_snapshots, rep_site_off, nE, npH, nT,
                        n_inst: int = 1, nHam: int = 1):
    """occ[g, k]: time-averaged state (0/1) of the k-th site of a replica over the
    snapshots in which that replica sat at grid point g (summed over grid
    instances, which share the topology), and n[g] the number of samples.
    state_snapshots: [n_snap, n_sites]; target_snapshots: [n_snap, n_rep, 4]."""
    S = np.asarray(state_snapshots)
    T = np.asarray(target_snapshots)
    off = np.asarray(rep_site_off)
    n_rep = off.size - 1
    k_sites = int(off[1] - off[0])
    G = nE * npH * nT * nHam
    tot = np.zeros((G, k_sites))
    n = np.zeros(G)
    g = grid_index(T, npH, nT, nHam)
    for r in range(n_rep):
        st = S[:, off[r]:off[r + 1]]
        np.add.at(tot, g[:, r], st)
        np.add.at(n, g[:, r], 1)
    return tot / np.maximum(n, 1)[:, None], n


# -------------------------------------------------------------- fits
def _linear_fit(x, y, w=None):
    x, y = np.asarray(x, float), np.asarray(y, float)
    w = np.ones_like(x) if w is None else np.asarray(w, float)
    A = np.stack([x, np.ones_like(x)], axis=1) * np.sqrt(w)[:, None]
    coef, *_ = np.linalg.lstsq(A, y * np.sqrt(w), rcond=None)
    return coef  # slope, intercept


def fit_pka(pH, f_prot, n_samples=None, eps=1e-3):
    """Eq. 1, f = 1 / (1 + 10^(n (pH - pKa))): linear fit of
    log10((1 - f)/f) = n pH - n pKa over points with eps < f < 1 - eps, weighted
    by the binomial variance of the logit.  Returns (pKa, n)."""
    pH, f = np.asarray(pH, float), np.asarray(f_prot, float)
    m = (f > eps) & (f < 1 - eps)
    if m.sum() < 2:
        raise ValueError("need at least two fractions strictly between 0 and 1")
    y = np.log10((1 - f[m]) / f[m])
    w = None if n_samples is None else np.asarray(n_samples, float)[m] * f[m] * (1 - f[m])
    slope, icpt = _linear_fit(pH[m], y, w)
    return -icpt / slope, slope


def fit_e0(E, f_red, T=300.0, n_samples=None, eps=1e-3):
    """Eq. 2 with v = 1, f = 1 / (1 + exp(n F (E - E0) / kT)): linear fit of
    ln((1 - f)/f) = (nF/kT) E - (nF/kT) E0.  Returns (E0 in V, n)."""
    E, f = np.asarray(E, float), np.asarray(f_red, float)
    m = (f > eps) & (f < 1 - eps)
    if m.sum() < 2:
        raise ValueError("need at least two fractions strictly between 0 and 1")
    y = np.log((1 - f[m]) / f[m])
    w = None if n_samples is None else np.asarray(n_samples, float)[m] * f[m] * (1 - f[m])
    slope, icpt = _linear_fit(E[m], y, w)
    c = FARADAY / (KB * T)
    return -icpt / slope, slope / c


# ------------------------------------------------------------ eqs. 6-8
def eq6_shift(pka_red, pka_oxi, T=300.0, v=1):
    """Eq. 6: E0_prot - E0_deprot (V) from the per-site pKa shifts."""
    return KB * T * LN10 / (v * FARADAY) * float(np.sum(np.asarray(pka_red) - np.asarray(pka_oxi)))


def eq7_e0(pH, e0_prot, pka_red, pka_oxi, T=300.0, v=1):
    """Eq. 7: pH-dependent E0 (V) of one redox site next to pH sites i."""
    pH = np.asarray(pH, float)
    s = 0.0
    for pr, po in zip(np.atleast_1d(pka_red), np.atleast_1d(pka_oxi)):
        s = s + np.log((10.0 ** -pr + 10.0 ** -pH) / (10.0 ** -po + 10.0 ** -pH))
    return e0_prot + KB * T / (v * FARADAY) * s


def eq8_sum_pka(E, e0_prot, e0_deprot, sum_pka_red, T=300.0, v=1):
    """Eq. 8: E-dependent sum of the sites' pKa values."""
    E = np.asarray(E, float)
    kT = KB * T
    a = -v * FARADAY * e0_prot / kT
    b = -v * FARADAY * e0_deprot / kT
    c = -FARADAY * E / kT
    # log10((e^a + e^c) / (e^b + e^c)) evaluated stably
    return sum_pka_red + (np.logaddexp(a, c) - np.logaddexp(b, c)) / LN10
