"""Benchmark: batched GB energy+force pair-interactions/s on one MI355X.

Workload (default): the 3-D E,T,pH replica-exchange batch -- 192 replicas
(8 E x 4 T x 6 pH) of one 1,024-atom synthetic system -- advanced by md_step:
every step evaluates the Born radii, GB + Coulomb + LJ energy and forces with
the chain rule, the Langevin update, titration attempts every 10 steps and an
exchange attempt every 100 steps, all on the device.  A step processes
192 * 1024 * 1023 / 2 = 100,564,992 pair interactions.

Prints one JSON line (see the keys below).  Timing: W untimed warm-up steps,
then K steps between two synchronizations.  Inside the timed region the
library records HIP events on the launch stream around every launch of the
dominant pair kernel (the slowest pass in the autotuner's timing), which gives
the roofline entry; the three passes side by side come from a short run after
the timed region.

--gpus N with N > 1 is refused: the batch runs on one GPU.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Algorithmic FLOPs per unordered pair (FMA = 2; add, sub, mul, div, sqrt,
# rsqrt, exp, log = 1; compare, select, min/max, abs = 0; per-atom
# precomputations not counted), from the closed forms of each pass:
FLOP_BORN = 49     # distance + both HCT descreening terms and their accumulation
FLOP_ENERGY = 64   # Coulomb + GB + LJ energies, direct forces, dE/dR_i and dE/dR_j
FLOP_CHAIN = 55    # distance + both dh/dr terms, chain coefficients, forces
FLOP_PAIR = FLOP_BORN + FLOP_ENERGY + FLOP_CHAIN
PEAK_FP32_TFLOPS = 157.3   # MI355X dense FP32 vector peak (256 CU x 2.4 GHz x 256 FLOP/clk)
PAPER_CONTEXT = {
    "source": "Table 1: pmemd.cuda.MPI E,pH,T-REMD, 237-atom NAcMP8 system, GB igb=2, "
              "one NVIDIA Tesla K20X per replica, 216 replicas",
    "ns_per_day_per_replica": 181, "dt_fs": 2,
    "step_ms_per_replica": 1e6 / (181e6 / 2.0 / 86400.0) / 1000.0,
    "pairs_per_s_per_gpu_upper_bound": 237 * 236 / 2 * 181e6 / 2.0 / 86400.0,
}


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=200)
    p.add_argument("--warmup", type=int, default=20)
    p.add_argument("--config", type=int, default=2)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-plain", action="store_true")
    p.add_argument("--graph", action="store_true", help="time the captured-graph path instead")
    p.add_argument("--cpu-sample-replicas", type=int, default=0)
    p.add_argument("--profile-only", action="store_true",
                   help="short run for rocprofv3: warm-up and a few timed steps, no baselines")
    p.add_argument("--copy-calibration", action="store_true",
                   help="also run a plain 256 MiB device copy (HBM counter calibration)")
    return p.parse_args()


# The files that hold the pair kernels' device code: the kernels, the device
# helpers, the far-field fits and the work-list layout.
PAIR_SOURCES = ("pair_kernels.hip", "gbr_device.h", "hct_poly.h", "pair_list.h")


def source_hash():
    """Hash of the pair kernels' sources, to tell whether a stored counter
    profile was taken on the current pair kernels."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1809_07726_amd", "csrc")
    for name in PAIR_SOURCES:
        h.update(open(os.path.join(csrc, name), "rb").read())
    return h.hexdigest()[:16]


def traffic_from_profile(kernel, workload):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary (taken on the 192 x 1,024 batch), if it was taken on the current
    kernel sources and the workload is that batch; else None."""
    if not workload.startswith("c2_"):
        return None
    path = os.path.join(ROOT, "profiles", "pair_kernels_c2_hbm_traffic.json")
    if not os.path.exists(path):
        return None
    d = json.load(open(path))
    if d.get("source_hash") != source_hash():
        return None
    k = d.get("kernels", {}).get(kernel)
    return None if k is None else k.get("bytes_per_launch")


def tuned_summary(tuned):
    return {"waves_per_group_x_groups_per_cu": tuned["shape"],
            "i_atoms_per_lane_born_energy_chain": tuned["blocking"], "split_den": tuned["split"]}


def pair_counts(b, cut):
    """Unordered pairs per replica: all of them, or those closer than cut."""
    off = b["atom_off"]
    n = np.diff(off).astype(np.int64)
    if not cut:
        return n * (n - 1) // 2
    from scipy.spatial import cKDTree
    out = np.zeros(n.size, np.int64)
    for r in range(n.size):
        tree = cKDTree(np.asarray(b["xyz"][off[r]:off[r + 1]], np.float64))
        out[r] = (tree.count_neighbors(tree, np.nextafter(cut, 0.0)) - n[r]) // 2
    return out


def cpu_model() -> str:
    """The host CPU's model name (from /proc/cpuinfo), or "unknown"."""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(b, n_rep_sample, gpu_ref=None, ext=None, rep_pairs=None, min_s=10.0, budget_s=20.0):
    """The FP64 oracle (as it stands) on a bounded sample of the same workload:
    full E+F gradient evaluations of successive replicas (cycling through the
    batch) until at least min_s seconds of CPU work, stopping at budget_s or
    after n_rep_sample evaluations (0: no count limit).  With gpu_ref = (E, F),
    the GPU's energies [n_rep, 5] and forces [N, 3] at the same inputs, also
    returns the GPU's error against FP64 on the replicas evaluated."""
    import oracle
    gb = oracle.obc2(**(ext or {}))
    off = b["atom_off"]
    t0 = time.perf_counter()
    pairs = 0
    done = 0
    first = {}
    while True:
        el = time.perf_counter() - t0
        if el > budget_s or (n_rep_sample and done >= n_rep_sample) or (el >= min_s and done >= 1):
            break
        r = done % b["n_rep"]
        done += 1
        a, c = off[r], off[r + 1]
        E, gx, _, _ = oracle.gradient(b["xyz"][a:c], b["q"][a:c], b["rho"][a:c], b["screen"][a:c],
                                      b["sigma"][a:c], b["eps"][a:c], gb)
        if r not in first:
            first[r] = (E, gx)
        n = c - a
        pairs += int(rep_pairs[r]) if rep_pairs is not None else n * (n - 1) // 2
    dt = time.perf_counter() - t0
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    cores = min(cores, os.cpu_count() or cores)
    sizes = np.diff(off)
    size_txt = (f"{sizes[0]} atoms" if np.all(sizes == sizes[0]) else f"{sizes.min()}..{sizes.max()} atoms")
    out = {"value": pairs / dt, "unit": "pair-interactions/s", "cores": cores, "kind": "oracle",
           "cpu_model": cpu_model(), "host_cpus": os.cpu_count(),
           "sample": f"{done} replica evaluations ({done / b['n_rep']:.2f} passes over the "
                     f"{b['n_rep']} replicas of {size_txt}): one FP64 Born-radii + energy + "
                     f"analytic-gradient evaluation each ({dt:.1f} s)"}
    err = None
    if gpu_ref is not None and first:
        Eg, Fg = gpu_ref
        e_rel, gb_rel, f_rms = [], [], []
        for r, (E, gx) in first.items():
            a, c = off[r], off[r + 1]
            e_rel.append(abs(Eg[r, 4] - E.sum()) / abs(E.sum()))
            gb_rel.append(abs(Eg[r, 0] - E[0]) / abs(E[0]))
            f_rms.append(float(np.sqrt(((Fg[a:c] + gx) ** 2).sum() / (gx ** 2).sum())))
        err = {"replicas": len(first), "state": "the synthetic starting coordinates",
               "energy_rel_max": max(e_rel), "e_gb_rel_max": max(gb_rel),
               "force_rms_rel_max": max(f_rms)}
    return out, err


def _progress(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "--gpus must be 1: the replica batch runs on one GPU "
                                   "and is not sharded across GPUs"}))
        sys.exit(2)
    import torch
    from paper_1809_07726_amd import synth
    from paper_1809_07726_amd.gb import MD, Context, DeviceBatch, reference_energies
    from paper_1809_07726_amd.tune import autotune

    import paper_1809_07726_amd._capi as A
    torch.cuda.set_device(0)
    b = synth.make_config(args.config)
    w = synth.CONFIGS[args.config]
    ext = {k: w.extra[k] for k in ("kappa", "cut", "rgbmax") if k in w.extra}
    params = A.obc2(**ext)
    b["G_ref"] = reference_energies(b, params)
    ctx = Context(b["atom_off"], params)
    dev = DeviceBatch.from_numpy(b)
    md = MD(ctx, dev, b, seed=w.dyn_seed)
    # a pair interaction: an unordered pair of one replica that the evaluation
    # counts (with a cutoff: the pairs within it at the starting coordinates)
    rep_pairs = pair_counts(b, ext.get("cut", 0.0))
    n_pairs = int(rep_pairs.sum())
    stream = torch.cuda.current_stream()

    _progress(f"{w.name}: {b['n_rep']} replicas, {n_pairs} pairs per step; autotuning")
    tuned = autotune(ctx, dev.t)
    _progress(f"tuned {tuned}; warmup")
    # the GPU's energies and forces at the starting coordinates: the cpu_baseline
    # leg compares them with the FP64 oracle on the replicas it evaluates
    t = dev.t
    R0, dR0, _ = ctx.born_radii(t["xyz"], t["rho"], t["screen"], want_psi=False)
    f0, e0, _, _ = ctx.energy_forces(t["xyz"], t["q"], t["rho"], t["screen"], t["sigma"], t["eps"], R0, dR0)
    gpu_ref = (ctx.energies(e0).cpu().numpy(),
               (f0.cpu().numpy() * 2.0 ** -40).reshape(3, -1).T.copy())
    ctx.check()
    md.run(0, init_forces=True)
    md.run(args.warmup if not args.profile_only else 3, graph=args.graph)
    torch.cuda.synchronize()
    ctx.check()
    K = args.steps if not args.profile_only else 5
    # Only the dominant pair pass (slowest in the autotuner's own timing) is
    # bracketed by HIP events inside the timed region: every event pair costs
    # a few microseconds of queue time between kernels.
    flops = {"born_pair": FLOP_BORN, "energy_pair": FLOP_ENERGY, "chain_pair": FLOP_CHAIN}
    dom = max(tuned["ms"], key=lambda k: tuned["ms"][k])
    _progress(f"timing {K} steps (events on {dom})")
    ctx.set_timing(not args.graph, (dom,))
    ctx.get_timing()                       # reset
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    md.run(K, graph=args.graph)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    timing = ctx.get_timing() if not args.graph else {}
    ctx.set_timing(False)
    ctx.check()
    if args.profile_only:
        if args.copy_calibration:
            x = torch.empty(64 * 1024 * 1024, dtype=torch.float32, device="cuda")
            y = torch.empty_like(x)
            for _ in range(3):
                y.copy_(x)
            torch.cuda.synchronize()
        print(json.dumps({"profile_only": True, "workload": w.name, "steps": K, "ms_per_step": 1000 * dt / K,
                          "tuned": tuned_summary(tuned), "source_hash": source_hash()}))
        return

    value = K * n_pairs / dt
    ms_step = 1000.0 * dt / K
    roofline = None
    ms, cnt = timing.get(dom, (0.0, 0))
    if cnt:
        avg = ms / cnt
        ach = flops[dom] * n_pairs / (avg * 1e-3) / 1e12
        traffic = traffic_from_profile(dom, w.name)
        roofline = {"bound": "alu", "kernel": dom, "achieved": ach, "peak": PEAK_FP32_TFLOPS,
                    "unit": "TFLOP/s", "frac": ach / PEAK_FP32_TFLOPS,
                    "traffic": traffic, "hbm_gbs": (traffic / (avg * 1e-3) / 1e9 if traffic else None),
                    "avg_launch_ms": avg, "launches": cnt,
                    "flop_per_pair": flops[dom], "pairs_per_launch": n_pairs}
    # the three pair passes side by side, from a short run after the timed region
    n_break = 20
    ctx.set_timing(True, tuple(flops))
    ctx.get_timing()
    md.run(n_break)
    torch.cuda.synchronize()
    tb = ctx.get_timing()
    ctx.set_timing(False)
    per_kernel = {}
    for k in flops:
        ms_k, cnt_k = tb.get(k, (0.0, 0))
        if cnt_k:
            avg_k = ms_k / cnt_k
            per_kernel[k] = {"avg_ms": avg_k, "launches": cnt_k,
                             "tflops": flops[k] * n_pairs / (avg_k * 1e-3) / 1e12}
    # the same number of steps replayed from the captured per-step graphs; a
    # warm-up of one exchange period captures the step kinds first
    graph_ms = None
    if not args.graph:
        md.run(max(w.ex_every, w.mc_every, 1), graph=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        md.run(K, graph=True)
        torch.cuda.synchronize()
        graph_ms = 1000.0 * (time.perf_counter() - t0) / K
        ctx.check()
    pair_ms = sum(v["avg_ms"] for v in per_kernel.values())
    all_pairs_tflops = FLOP_PAIR * n_pairs / (pair_ms * 1e-3) / 1e12 if pair_ms else None

    _progress(f"{ms_step:.4f} ms/step; batched vs per-replica evaluation")
    # batched vs per-replica plain E+F evaluation (same kernels, one launch sequence per replica)
    evals = {}
    t = dev.t
    R, dR, psi = ctx.born_radii(t["xyz"], t["rho"], t["screen"])
    for _ in range(3):
        R, dR, _ = ctx.born_radii(t["xyz"], t["rho"], t["screen"], want_psi=False)
        ctx.energy_forces(t["xyz"], t["q"], t["rho"], t["screen"], t["sigma"], t["eps"], R, dR)
    torch.cuda.synchronize()
    n_eval = 20
    t0 = time.perf_counter()
    for _ in range(n_eval):
        R, dR, _ = ctx.born_radii(t["xyz"], t["rho"], t["screen"], want_psi=False)
        ctx.energy_forces(t["xyz"], t["q"], t["rho"], t["screen"], t["sigma"], t["eps"], R, dR)
    torch.cuda.synchronize()
    evals["batched_eval_ms"] = 1000 * (time.perf_counter() - t0) / n_eval
    if not args.no_plain:
        off = b["atom_off"]
        N = ctx.n_atoms
        # one single-replica context per distinct replica size; the launch tuned
        # for the largest size is used for all of them
        sizes = np.diff(off).astype(int)
        pctx = {int(n): Context(np.array([0, n], np.int32), params) for n in np.unique(sizes)}
        reps = []
        for r in range(b["n_rep"]):
            a, c = off[r], off[r + 1]
            sl = lambda key: t[key][a:c].contiguous()
            xyz = torch.stack([t["xyz"][a:c], t["xyz"][N + a:N + c], t["xyz"][2 * N + a:2 * N + c]]).reshape(-1).contiguous()
            reps.append((pctx[int(c - a)], xyz, sl("q"), sl("rho"), sl("screen"), sl("sigma"), sl("eps")))
        def plain_pass():
            for pc, xyz, q, rho, scr, sig, eps in reps:
                R1, dR1, _ = pc.born_radii(xyz, rho, scr, want_psi=False)
                pc.energy_forces(xyz, q, rho, scr, sig, eps, R1, dR1)
        big = int(np.argmax(sizes))
        pt = autotune(reps[big][0], {"xyz": reps[big][1], "q": reps[big][2], "rho": reps[big][3],
                                     "screen": reps[big][4], "sigma": reps[big][5], "eps": reps[big][6]})
        for pc in pctx.values():
            pc.set_split(pt["split"])
            pc.set_launch(*pt["shape"])
            pc.set_blocking(*pt["blocking"])
        plain_pass()
        torch.cuda.synchronize()
        n_plain = 3
        t0 = time.perf_counter()
        for _ in range(n_plain):
            plain_pass()
        torch.cuda.synchronize()
        evals["plain_eval_ms"] = 1000 * (time.perf_counter() - t0) / n_plain
        evals["speedup_batched_vs_plain"] = evals["plain_eval_ms"] / evals["batched_eval_ms"]
        for pc in pctx.values():
            pc.close()
    evals["batched_eval_pairs_per_s"] = n_pairs / (evals["batched_eval_ms"] * 1e-3)
    if "plain_eval_ms" in evals:
        evals["plain_eval_pairs_per_s"] = n_pairs / (evals["plain_eval_ms"] * 1e-3)

    cpu, err64 = None, None
    if not args.no_cpu_baseline:
        _progress("oracle CPU baseline")
        cpu, err64 = cpu_baseline(b, args.cpu_sample_replicas, gpu_ref, ext, rep_pairs)

    sizes = np.diff(b["atom_off"]).astype(int)
    atoms_per_replica = (int(sizes[0]) if np.all(sizes == sizes[0]) else
                         {"min": int(sizes.min()), "max": int(sizes.max()), "total": int(sizes.sum())})
    out = {
        "metric": "GB energy+force pair-interactions/s, batched replicas vs per-replica plain",
        "value": value, "unit": "pair-interactions/s", "n_gpus": 1, "steps": K,
        "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w.name, "replicas": int(b["n_rep"]), "atoms_per_replica": atoms_per_replica,
                   "grid": f"{len(w.E_vals)} E x {len(w.T_vals)} T x {len(w.pH_vals)} pH",
                   "gb_extensions": ext or None,
                   "pairs_per_step": n_pairs, "mc_every": w.mc_every,
                   "ex_every": w.ex_every, "graph": bool(args.graph),
                   "accumulation": "int64 fixed point (forces 2^-40, energies 2^-32)",
                   "tuned": tuned_summary(tuned)},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "error_vs_fp64": err64,
        "pair_kernels": per_kernel,
        "graph_ms_per_step": graph_ms,
        "pair_kernels_note": f"all three passes timed with events over {n_break} steps after the timed region",
        "all_pair_passes_tflops": all_pairs_tflops,
        "eval": evals,
        "paper_context": PAPER_CONTEXT,
        "source_hash": source_hash(),
    }
    print(json.dumps(out))
    ctx.close()


if __name__ == "__main__":
    main()
