"""Seeded synthetic inputs for the batched GB / C(pH,E)MD / REMD path.

This module is the only code shared by the HIP path's tests and benchmark and
by the CPU oracle: it draws geometry, parameters, titratable-site tables and
replica grids, and holds none of the method's arithmetic (no Born radii, no
energies, no reference energies; those are computed by whichever side consumes
the inputs).  Everything is numpy with an explicit seed.

Stand-in for the paper's system.  The paper's NAcMP8 + histidine peptide
(237 atoms, FF99SB with heme charges; Calculation details) is not available,
so systems are atoms on a 3.0 A cubic lattice with uniform jitter, random
charges and radii drawn from the distributions listed in ``CONFIGS``; a
titratable residue is modelled as a small cluster of neighbouring atoms whose
charges change between two states (a pH site gains +1 e when protonated, a
redox site gains -1 e when reduced), mirroring how the paper represents
protonation/redox states as atomic charge sets.

Every per-atom float array is produced in float32 so that the GPU path and the
oracle consume bit-identical values (the oracle promotes them exactly).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

PH_SITE, REDOX_SITE = 0, 1
DIM_E, DIM_PH, DIM_T, DIM_H = 0, 1, 2, 3


@dataclass(frozen=True)
class Workload:
    name: str
    n_atoms: tuple          # per system (or a range for the uneven batch)
    replicas_per_system: int
    n_systems: int
    n_ph: int               # pH sites per system (or -1: one per 200 atoms, alternating)
    n_redox: int
    E_vals: tuple           # V
    pH_vals: tuple
    T_vals: tuple           # K
    dim_order: tuple
    steps: int
    mc_every: int
    ex_every: int
    per_replica_jitter: bool
    geo_seed: int
    dyn_seed: int
    extra: dict = field(default_factory=dict)


def _lin(a, b, n):
    return tuple(float(v) for v in np.linspace(a, b, n))


# The workloads: a single-replica correctness system, the 2-D E,pH and 3-D
# E,T,pH replica grids, a differentiation batch, an uneven batch, and one large
# system with salt and cutoffs.
CONFIGS = {
    0: Workload("c0_single_256", (256,), 1, 1, 1, 1, (-0.2,), (6.5,), (300.0,), (DIM_E,),
                1000, 10, 0, False, 1000, 2000),
    1: Workload("c1_EpH_48x1024", (1024,), 48, 1, 5, 1, _lin(-0.35, 0.05, 8), _lin(4.0, 9.0, 6),
                (300.0,), (DIM_E, DIM_PH), 10000, 10, 100, False, 1001, 2001),
    2: Workload("c2_ETpH_192x1024", (1024,), 192, 1, 5, 1, _lin(-0.35, 0.05, 8), _lin(4.0, 9.0, 6),
                (300.0, 315.0, 330.0, 345.0), (DIM_E, DIM_T, DIM_PH), 10000, 10, 100, False,
                1002, 2002),
    3: Workload("c3_grad_16x4096", (4096,), 16, 1, 1, 1, (-0.2,), (6.5,), (300.0,), (DIM_E,),
                0, 10, 0, True, 1003, 2003),
    4: Workload("c4_uneven_64sys", (500, 20000), 4, 64, -1, -1, (-0.2,), (5.0, 6.0, 7.0, 8.0),
                (300.0,), (DIM_PH,), 0, 10, 100, False, 1004, 2004),
    # beyond the all-pairs regime: salt and cutoffs on one large system whose
    # atoms come in compact 64-atom blocks (the pair passes pack the atoms near each block)
    5: Workload("c5_salt_cutoff_1x100k", (100000,), 1, 1, -1, -1, (-0.2,), (7.0,), (300.0,), (DIM_E,),
                0, 10, 0, False, 1005, 2005,
                extra={"kappa": 0.1, "cut": 12.0, "rgbmax": 15.0, "blocked": True}),
}

PH_SITE_ATOMS = 4       # atoms per pH site; protonation adds 1/4 e to each
REDOX_SITE_ATOMS = 8    # atoms per redox site; reduction adds -1/8 e to each
LATTICE = 3.0           # A
JITTER = 0.3            # A, uniform per coordinate
K_TETHER = 5.0          # kcal/(mol A^2)
MASS = 12.01            # amu
DT = 0.001              # ps (1 fs)
GAMMA = 10.0            # 1/ps
PKA_REF = 6.5
E0_REF = -0.2           # V


def lattice_sites(n_atoms: int, spacing: float = LATTICE, blocked: bool = False):
    """First n_atoms sites of an n^3 cubic lattice (n = ceil(cbrt N)), x fastest;
    with ``blocked`` the sites are ordered by 4 x 4 x 4 blocks first (blocks x
    fastest, then within a block x fastest), so that 64 consecutive atoms fill
    one compact cube."""
    n = 1
    while n ** 3 < n_atoms:
        n += 1
    m = np.arange(n ** 3 if blocked else n_atoms)
    ijk = np.stack([m % n, (m // n) % n, m // (n * n)], axis=1)
    if blocked:
        nb = (n + 3) // 4
        b, w = ijk // 4, ijk % 4
        key = ((b[:, 2] * nb + b[:, 1]) * nb + b[:, 0]) * 64 + (w[:, 2] * 4 + w[:, 1]) * 4 + w[:, 0]
        ijk = ijk[np.argsort(key, kind="stable")][:n_atoms]
    return ijk, ijk.astype(np.float64) * spacing


def draw_system(n_atoms: int, seed: int, n_ph: int, n_redox: int, alternate=False, blocked=False):
    """One system: jittered lattice, per-atom parameters and site clusters.

    Sites are disjoint clusters: for each site a random unused atom is drawn and
    the k unused atoms whose lattice sites are nearest to its lattice site
    (ties broken by index) form the site.  With ``alternate`` the site types
    alternate pH, redox, pH, ... (n_ph + n_redox sites in total); otherwise all
    pH sites come first."""
    rng = np.random.default_rng(seed)
    ijk, x0 = lattice_sites(n_atoms, blocked=blocked)
    xyz = x0 + rng.uniform(-JITTER, JITTER, size=x0.shape)
    q = rng.normal(0.0, 0.3, size=n_atoms)
    q -= q.mean()
    rho = rng.uniform(1.2, 2.0, size=n_atoms)
    scr = rng.uniform(0.7, 0.9, size=n_atoms)
    sig = rng.uniform(2.5, 3.5, size=n_atoms)
    eps = rng.uniform(0.05, 0.2, size=n_atoms)
    n_sites = n_ph + n_redox
    if alternate:
        types = [PH_SITE if k % 2 == 0 else REDOX_SITE for k in range(n_sites)]
    else:
        types = [PH_SITE] * n_ph + [REDOX_SITE] * n_redox
    used = np.zeros(n_atoms, dtype=bool)
    sites = []
    f32 = lambda a: np.asarray(a, dtype=np.float32)
    q32 = f32(q)
    for t in types:
        k = PH_SITE_ATOMS if t == PH_SITE else REDOX_SITE_ATOMS
        free = np.flatnonzero(~used)
        if free.size < k:
            raise ValueError("not enough atoms for the requested sites")
        c = free[rng.integers(free.size)]
        d2 = ((ijk[free] - ijk[c]) ** 2).sum(axis=1)
        order = np.lexsort((free, d2))
        atoms = np.sort(free[order[:k]])
        used[atoms] = True
        s0 = q32[atoms].astype(np.float64)
        delta = (1.0 if t == PH_SITE else -1.0) / k
        s1 = f32(s0 + delta).astype(np.float64)
        sites.append({"type": t, "atoms": atoms, "q_states": np.stack([s0, s1], axis=1),
                      "nH": [0, 1] if t == PH_SITE else [0, 0],
                      "ne": [0, 0] if t == PH_SITE else [0, 1],
                      "ref": PKA_REF if t == PH_SITE else E0_REF})
    return {"xyz": f32(xyz), "x0": f32(x0), "q": q32, "rho": f32(rho), "screen": f32(scr),
            "sigma": f32(sig), "eps": f32(eps), "mass": np.full(n_atoms, MASS, np.float32),
            "sites": sites}


def jitter_copy(sysd: dict, seed: int):
    """Same topology and parameters, independent jitter of the lattice."""
    rng = np.random.default_rng(seed)
    out = dict(sysd)
    x0 = sysd["x0"].astype(np.float64)
    out["xyz"] = (x0 + rng.uniform(-JITTER, JITTER, size=x0.shape)).astype(np.float32)
    return out


def assemble(systems: list, reps_per_system: int, E_vals, pH_vals, T_vals, dim_order,
             per_replica: list | None = None, H_scale=(1.0,), **md):
    """Flatten replicas of each system back to back and build the site tables
    and the replica grid (one grid instance per system; replica k of a system
    starts at grid point k, g = ((iE * npH + ipH) * nT + iT) * nHam + iH, with
    H_scale the scales of the GB + Coulomb + LJ energy at the Hamiltonian
    levels).

    ``per_replica`` optionally gives a distinct system dict (same topology) for
    every replica."""
    nE, npH, nT, nHam = len(E_vals), len(pH_vals), len(T_vals), len(H_scale)
    G = nE * npH * nT * nHam
    if reps_per_system != G:
        raise ValueError("replicas per system must equal the grid size")
    reps = per_replica or [s for s in systems for _ in range(reps_per_system)]
    sizes = [r["q"].size for r in reps]
    atom_off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int32)
    cat = lambda key: np.concatenate([r[key] for r in reps])
    out = {k: cat(k) for k in ("xyz", "x0", "q", "rho", "screen", "sigma", "eps", "mass")}
    out["atom_off"] = atom_off
    out["n_rep"] = len(reps)
    # sites: a site dict gives one charge column and one (nH, ne) entry per
    # state; the tables are padded to the batch's largest state count
    ms = max([2] + [len(s["nH"]) for rd in reps for s in rd["sites"]])
    site_off, site_atoms, site_type, n_states, state_q = [0], [], [], [], []
    state_nH, state_ne, ref_value, rep_site_off, site_rep = [], [], [], [0], []
    for r, rd in enumerate(reps):
        for s in rd["sites"]:
            k = len(s["nH"])
            qs = np.asarray(s["q_states"], np.float64).reshape(len(s["atoms"]), k)
            site_atoms.extend((s["atoms"] + atom_off[r]).tolist())
            site_off.append(len(site_atoms))
            site_type.append(s["type"])
            n_states.append(k)
            state_q.append(np.pad(qs, ((0, 0), (0, ms - k))))
            state_nH.extend(list(s["nH"]) + [0] * (ms - k))
            state_ne.extend(list(s["ne"]) + [0] * (ms - k))
            ref_value.append(s["ref"])
            site_rep.append(r)
        rep_site_off.append(len(site_type))
    out.update({
        "n_sites": len(site_type), "max_states": ms,
        "site_off": np.asarray(site_off, np.int32), "site_atoms": np.asarray(site_atoms, np.int32),
        "site_type": np.asarray(site_type, np.int32), "n_states": np.asarray(n_states, np.int32),
        "state_q": (np.concatenate(state_q).reshape(-1) if state_q else np.zeros(0)).astype(np.float64),
        "state_nH": np.asarray(state_nH, np.int32), "state_ne": np.asarray(state_ne, np.int32),
        "ref_value": np.asarray(ref_value, np.float64),
        "rep_site_off": np.asarray(rep_site_off, np.int32), "site_rep": np.asarray(site_rep, np.int32),
        "site_state": np.zeros(len(site_type), np.int32),
        "G_ref": np.zeros(ms * len(site_type), np.float64),  # filled by the consumer
    })
    # grid
    n_inst = len(systems) if per_replica is None else len(reps) // reps_per_system
    g = np.arange(out["n_rep"]) % G
    out["target_idx"] = np.stack([g // (npH * nT * nHam), (g // (nT * nHam)) % npH,
                                  (g // nHam) % nT, g % nHam], axis=1).astype(np.int32)
    out["grid_rep"] = np.arange(out["n_rep"], dtype=np.int32)
    out.update({"n_inst": n_inst, "E_vals": np.asarray(E_vals, np.float64),
                "pH_vals": np.asarray(pH_vals, np.float64), "T_vals": np.asarray(T_vals, np.float64),
                "H_scale": np.asarray(H_scale, np.float64), "dim_order": list(dim_order)})
    out["v"] = np.zeros_like(out["xyz"])
    out.update({"k_tether": K_TETHER, "dt": DT, "gamma_ps": GAMMA, "mc_every": 10, "ex_every": 0})
    out.update(md)
    return out


def make_config(idx: int, *, n_atoms: int | None = None, n_rep: int | None = None,
                n_systems: int | None = None, per_replica_jitter: bool | None = None,
                seed: int | None = None):
    """Synthetic batch for workload ``idx`` (0..5); the keyword arguments
    shrink it for tests (fewer atoms, replicas or systems) while keeping the
    workload's structure and distributions."""
    w = CONFIGS[idx]
    seed = w.geo_seed if seed is None else seed
    prj = w.per_replica_jitter if per_replica_jitter is None else per_replica_jitter
    md = {"mc_every": w.mc_every, "ex_every": w.ex_every, "steps": w.steps, "dyn_seed": w.dyn_seed,
          "workload": w.name}
    if idx == 4:
        nsys = n_systems or w.n_systems
        rng = np.random.default_rng(seed)
        lo, hi = w.n_atoms
        sizes = np.exp(rng.uniform(math.log(lo), math.log(hi), size=nsys)).round().astype(int)
        if n_atoms is not None:
            sizes = np.minimum(sizes, n_atoms)
        systems = []
        for s, n in enumerate(sizes):
            ns = max(1, int(round(n / 200)))
            n_ph = (ns + 1) // 2
            systems.append(draw_system(int(n), seed * 1000 + s, n_ph, ns - n_ph, alternate=True))
        return assemble(systems, w.replicas_per_system, w.E_vals, w.pH_vals, w.T_vals, w.dim_order,
                        **md)
    n = n_atoms or w.n_atoms[0]
    if w.n_ph < 0:                      # one site per 200 atoms, alternating pH / redox
        ns = max(1, int(round(n / 200)))
        base = draw_system(n, seed, (ns + 1) // 2, ns // 2, alternate=True,
                           blocked=w.extra.get("blocked", False))
    else:
        base = draw_system(n, seed, w.n_ph, w.n_redox, blocked=w.extra.get("blocked", False))
    G = len(w.E_vals) * len(w.pH_vals) * len(w.T_vals)
    total = w.replicas_per_system * w.n_systems
    if n_rep is not None:
        total = n_rep
    if total % G == 0:
        E_vals, pH_vals, T_vals = w.E_vals, w.pH_vals, w.T_vals
    else:
        # shrunk test batch: keep the grid's dimensions but fewer points
        E_vals, pH_vals, T_vals = _shrink_grid(w, total)
    G = len(E_vals) * len(pH_vals) * len(T_vals)
    n_inst = total // G
    if prj:
        reps = [jitter_copy(base, seed * 7919 + r) for r in range(total)]
        return assemble([base] * n_inst, G, E_vals, pH_vals, T_vals, w.dim_order,
                        per_replica=reps, **md)
    return assemble([base] * n_inst, G, E_vals, pH_vals, T_vals, w.dim_order, **md)


def _shrink_grid(w: Workload, total: int):
    """A smaller grid with the same dimensions whose size divides ``total``."""
    dims = [list(w.E_vals), list(w.pH_vals), list(w.T_vals)]
    while True:
        G = len(dims[0]) * len(dims[1]) * len(dims[2])
        if total % G == 0:
            return tuple(dims[0]), tuple(dims[1]), tuple(dims[2])
        k = int(np.argmax([len(d) for d in dims]))
        dims[k] = dims[k][:-1]


def isolated_sites(batch: dict):
    """For every site of replica 0 of each system: the site's own atoms as a
    stand-alone system (the 'reference compound' geometry), as index arrays
    into the batch.  Consumers compute the reference energies from these."""
    out = []
    for s in range(batch["n_sites"]):
        a, b = batch["site_off"][s], batch["site_off"][s + 1]
        out.append(batch["site_atoms"][a:b])
    return out
