#!/usr/bin/env python3
"""Benchmark of the docking screen on one MI355X.

Workload: one 96^3 pocket with 16 atom types (300 seeded protein atoms), 100k seeded
synthetic ligands (atom counts N(35, 10) clipped to [15, 70], Poisson(5) rotatable bonds
clipped to [0, 12]), 256 quaternions x 32 translations, 256 torsion steps, top-1000.

One step = the whole hot path over the library with inputs resident in HBM:
grid build -> ligand pack -> screen (rigid starts + greedy torsion sweeps + best pose)
-> top-k.  Prints one JSON line.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "ligands docked/sec and poses scored/sec on 1 MI355X; recall@top1% with surrogate"
PEAK_FP32_NONPACKED = 78.6e12  # 256 CU x 64 FMA lanes/clk x 2 FLOP x 2.4 GHz
# Algorithmic FLOP per lookup, in the units of the scope table: a rigid-start atom 48 (transform 18,
# interpolation about 30), a sweep lookup 36 (circle-form move 6, interpolation about 30).  The kernel's
# own instruction-level count (an FMA as 2) is 46 and 40; it is reported beside them.
FLOP_RIGID_ATOM = 48
FLOP_SWEEP_LOOKUP = 36
FLOP_RIGID_ATOM_KERNEL = 46    # rotation 18 + grid coordinates 6 + trilinear 21 + sum 1
FLOP_SWEEP_LOOKUP_KERNEL = 40  # circle position 12 + grid coordinates 6 + trilinear 21 + sum 1
BYTES_PER_LOOKUP = 32          # eight FP32 corners
COUNTERS = os.path.join(ROOT, "profiles", "screen_counters.json")
SCREEN_SRC = os.path.join(ROOT, "paper_2304_09953_amd", "csrc", "screen.hip")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def screen_source_hash():
    return hashlib.sha256(open(SCREEN_SRC, "rb").read()).hexdigest()[:16]


def counters():
    """The committed rocprofv3 counter summary of the screen, if it was taken on the current kernel
    source; otherwise None."""
    try:
        c = json.load(open(COUNTERS))
    except (OSError, ValueError):
        return None
    return c if c.get("screen_src_sha256_16") == screen_source_hash() else None


def traffic_from_counters():
    """HBM bytes per screen launch from the counter summary, or None."""
    c = counters()
    return None if c is None else c.get("hbm_bytes_per_launch")


def _pmc(csv_dir, counter, kernel):
    """Per-dispatch values of one counter for one kernel, from a rocprofv3 --pmc CSV directory."""
    import csv
    import glob
    vals = {}
    for f in glob.glob(os.path.join(csv_dir, "*counter_collection.csv")):
        for r in csv.DictReader(open(f)):
            if r["Counter_Name"] == counter and r["Kernel_Name"] == kernel:
                vals[int(r["Dispatch_Id"])] = vals.get(int(r["Dispatch_Id"]), 0.0) + float(r["Counter_Value"])
    return [vals[k] for k in sorted(vals)]


def summarize_counters(out_dir):
    """Writes the counter summary (profiles/screen_counters.json) from the rocprofv3 --pmc runs
    listed in its "commands" (their CSV directories under out_dir)."""
    d = lambda name: os.path.join(out_dir, name)  # noqa: E731
    one = lambda name, counter, kernel="k_screen": _pmc(d(name), counter, kernel)[0]  # noqa: E731
    fetch, write = one("pmc_fetch", "FETCH_SIZE"), one("pmc_write", "WRITE_SIZE")
    cf = one("pmc_copy_fetch", "FETCH_SIZE", "__amd_rocclr_copyBuffer")
    cw = one("pmc_copy_write", "WRITE_SIZE", "__amd_rocclr_copyBuffer")
    ff, fw = (1 << 20) / cf, (1 << 20) / cw  # KiB counted for a 1 GiB copy
    req = one("pmc_req", "TCP_TCC_READ_REQ_sum")
    # bytes per L1-to-L2 request: the cache-resident read kernel's known bytes over its requests
    # (its three timed dispatches: 2048 blocks x 64 reads of 2 MiB)
    creq = _pmc(d("pmc_req_calib"), "TCP_TCC_READ_REQ_sum", "k_calib_read")[-3:]
    req_bytes = 3 * 2048 * 64 * (2 << 20) / sum(creq)
    valu = one("pmc_valu", "SQ_INSTS_VALU")
    gui = one("pmc_valu", "GRBM_GUI_ACTIVE")  # summed over the 8 XCDs
    hit, miss = one("pmc_req", "TCC_HIT_sum"), one("pmc_req", "TCC_MISS_sum")
    base = "cd /tmp && rocprofv3 --pmc {c} -T -f csv -d <out>/{d} -o {o} -- python3 -u <repo>/bench.py {a}"
    run1 = "--no-cpu-baseline --steps 1 --warmup 0"
    out = {
        "kernel": "k_screen",
        "workload": "pocket96-lib100k (100k ligands, 96^3 x 16 grid, 256 x 32 starts, 256 steps)",
        "screen_src_sha256_16": screen_source_hash(),
        "fetch_size_kib_per_launch": fetch, "write_size_kib_per_launch": write,
        "copy_reference": {"bytes": 1 << 30, "fetch_size_kib": cf, "write_size_kib": cw, "fetch_factor": ff,
                           "write_factor": fw},
        "hbm_bytes_per_launch": fetch * 1024 * ff + write * 1024 * fw,
        "l1_to_l2_requests_per_launch": req,
        "l1_to_l2_request_bytes": req_bytes,
        "l1_to_l2_bytes_per_launch": req * req_bytes,
        "l2_hit_rate": hit / (hit + miss),
        "l2_hits_per_launch": hit,
        "l2_misses_per_launch": miss,
        "valu_insts_per_launch": valu,
        "gpu_cycles_per_launch": gui / 8,
        "valu_busy": valu * 4 / (256 * 4) / (gui / 8),
        "commands": [base.format(c="FETCH_SIZE", d="pmc_fetch", o="fetch", a=run1),
                     base.format(c="WRITE_SIZE", d="pmc_write", o="write", a=run1),
                     base.format(c="FETCH_SIZE", d="pmc_copy_fetch", o="copy", a="--calibrate-copy 1024"),
                     base.format(c="WRITE_SIZE", d="pmc_copy_write", o="copy", a="--calibrate-copy 1024"),
                     base.format(c="TCP_TCC_READ_REQ_sum TCC_HIT_sum TCC_MISS_sum", d="pmc_req", o="req", a=run1),
                     base.format(c="TCP_TCC_READ_REQ_sum", d="pmc_req_calib", o="calib", a="--calibrate-peaks l2"),
                     base.format(c="SQ_INSTS_VALU GRBM_GUI_ACTIVE", d="pmc_valu", o="valu", a=run1),
                     f"python3 bench.py --summarize-counters <dir holding the CSV directories above>"],
        "note": ("FETCH_SIZE/WRITE_SIZE count L2-to-fabric traffic in KiB per dispatch (Infinity Cache hits "
                 "included), each scaled by what it reads for a plain 1 GiB device copy. L1-to-L2 requests are "
                 "scaled by the bytes per request of the cache-resident read kernel. VALU busy = VALU "
                 "instructions x 4 cycles (one wave64 instruction per SIMD every 4 cycles) over 1024 SIMDs x "
                 "the kernel's cycles."),
    }
    json.dump(out, open(COUNTERS, "w"), indent=1)
    print(json.dumps(out, indent=1))


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def cpu_sample(ligs, seed: int = 20240409):
    """Seeded, stratified order of library ligands for the CPU baseline: the largest ligand, one with
    the most torsions (12), one with none, the smallest, then seeded random draws."""
    import numpy as np
    n, b = ligs.n_atoms, ligs.n_rot
    first = [int(np.argmax(n)), int(np.flatnonzero(b == b.max())[0]), int(np.flatnonzero(b == 0)[0]),
             int(np.argmin(n))]
    rng = np.random.default_rng(seed)
    rest = [int(i) for i in rng.permutation(ligs.n_lig)[:256] if int(i) not in first]
    out = []
    for i in first + rest:
        if i not in out:
            out.append(i)
    return out


def cpu_baseline(W, ligs, budget_s):
    """The FP64 oracle on the host, on all threads OpenMP uses: a seeded stratified sample of the
    library (cpu_sample) docked one ligand at a time with the full search until budget_s seconds have
    passed (the four strata always run), then one ligand of median atom and torsion counts on one thread.  Rates are the
    sample's own; the library estimate rescales the sample's lookup rate by the library's mean
    lookups per ligand.  Grid build excluded."""
    import numpy as np

    import oracle
    pocket = W.pockets[0]
    log("cpu baseline: oracle grids")
    G = oracle.build_grids(pocket)
    cores = oracle.get_threads()
    Q, S = W.search.n_starts, W.search.n_steps
    n_rot = ligs.n_rot

    def lookups(idx):
        """Q T (n + (S - 1) sum_k |M_k|) per ligand: the oracle's own work (it also looks up each
        torsion's axis atom), moving sets from its own topology."""
        out = []
        for i in np.asarray(idx).tolist():
            tp = oracle.topology(ligs, i)
            out.append(Q * (ligs.n_atoms[i] + (S - 1) * float(tp["moving"].sum())) if tp["status"] == 0 else 0.0)
        return np.array(out)

    pose_count = lambda i: Q * (1 + int(n_rot[i]) * (S - 1))  # noqa: E731
    order = cpu_sample(ligs)
    done, poses, t0 = [], 0, time.perf_counter()
    for i in order:
        if len(done) >= 4 and time.perf_counter() - t0 >= budget_s:
            break
        oracle.dock(pocket, G, ligs, W.search, sel=np.array([i]))
        poses += pose_count(i)
        done.append(i)
        log(f"cpu baseline: {len(done)} ligands (last: n {ligs.n_atoms[i]}, B {n_rot[i]}), "
            f"{time.perf_counter() - t0:.1f} s")
    dt = time.perf_counter() - t0
    lib_lookups = float(lookups(np.random.default_rng(7).choice(ligs.n_lig, min(4000, ligs.n_lig),
                                                                 replace=False)).mean())
    samp_rate = float(lookups(done).sum()) / dt
    # a typical ligand: the first with the median atom count and the median torsion count
    med = int(np.flatnonzero((ligs.n_atoms == int(np.median(ligs.n_atoms))) & (n_rot == int(np.median(n_rot))))[0])
    oracle.set_threads(1)
    t1 = time.perf_counter()
    oracle.dock(pocket, G, ligs, W.search, sel=np.array([med]))
    dt1 = time.perf_counter() - t1
    oracle.set_threads(cores)
    log(f"cpu baseline: median ligand {med} on one thread, {dt1:.1f} s")
    return {"value": len(done) / dt, "unit": "ligands/s", "cores": cores, "kind": "oracle",
            "cpu_model": cpu_model(),
            "sample": (f"sample rate: {len(done)} ligands of a seeded stratified sample of the library (the "
                       "largest, one with 12 torsions, one with none, the smallest, then random draws), full "
                       "search, FP64 oracle, grid build excluded"),
            "sample_ids": done, "sample_n_atoms": [int(ligs.n_atoms[i]) for i in done],
            "sample_n_rot": [int(n_rot[i]) for i in done],
            "poses_per_sec": poses / dt, "seconds": round(dt, 2),
            "library_estimate_ligands_per_s": samp_rate / lib_lookups,
            "library_estimate_note": ("the sample's lookups per second over the mean lookups per ligand of 4000 "
                                      "seeded library ligands"),
            "one_core": {"value": 1 / dt1, "unit": "ligands/s", "poses_per_sec": pose_count(med) / dt1,
                         "sample": f"ligand {med} (median atom and torsion counts, n {int(ligs.n_atoms[med])}, "
                                   f"B {int(n_rot[med])}), full search, one OpenMP thread",
                         "seconds": round(dt1, 2)}}


def prefilter_bench(args):
    """Surrogate-filtered screening against plain docking on the same GPU."""
    import numpy as np

    from paper_2304_09953_amd import inputs as I
    from paper_2304_09953_amd import pipeline as P
    from paper_2304_09953_amd import prefilter as PF
    W = I.workload("pocket96-lib100k")
    pocket = W.pockets[0]
    dp = P.DevicePocket(pocket)
    ds = P.DeviceSearch(W.search)
    log(f"labels: docking {args.pf_train} training ligands")
    train = I.make_ligands(args.pf_train, W.dist, W.n_types, stream="train")
    sur = PF.train_surrogate(dp, ds, train, n_holdout=args.pf_train // 5, members=args.pf_members,
                             max_epochs=args.pf_epochs, log=log, linear_baseline=True)
    log(f"surrogate: {sur.metrics}")
    # ablation on the held-out docked ligands at the same budgets: the network, a linear model of the
    # same features fitted on the same training ligands, ligand size either way, random order
    hy = sur.holdout_true
    h_atoms = train.n_atoms[-len(hy):].astype(np.float64)
    abl_fracs = [0.01, 0.02, 0.03, 0.05, 0.1, 0.15, 0.2, 0.3]
    abl_keys = {"network": sur.holdout_pred, "linear": sur.holdout_linear, "smallest_first": h_atoms,
                "largest_first": -h_atoms, "random": np.random.default_rng(1).permutation(len(hy)).astype(np.float64)}
    ablation = {name: {f"{f:.3f}": v for f, v in PF.recall_curve(PF.ranks(k), hy, abl_fracs, len(hy)).items()}
                for name, k in abl_keys.items()}
    log(f"held-out ablation (recall of the true top 1 %): {ablation}")
    if args.pf_frac > 0:
        frac, how = args.pf_frac, "given"
    else:  # smallest fraction reaching the target recall (plus a margin) on the held-out docked ligands
        frac = PF.calibrate_fraction(sur.holdout_pred, sur.holdout_true, args.pf_target + args.pf_margin)
        how = (f"smallest with held-out recall >= {args.pf_target + args.pf_margin:.2f} "
               f"({len(sur.holdout_true)} held-out docked ligands)")
    log(f"docking the top {frac:.1%} by prediction ({how})")
    fixed = args.pf_fixed_frac
    cascade_ds, pools, cascade_how, cascade_top, candidates = None, (), None, 0, []
    tops = [int(v) for v in args.pf_cascade_tops.split(",") if v.strip()] if args.pf_cascade_tops else []
    if tops and fixed > 0:
        # cascade: the pool by prediction, docked with a smaller search budget, then the fixed top fraction of
        # the library by those scores docked in full.  For each budget (rigid starts swept) the pool is the
        # smallest reaching the target on the held-out ligands; the budget with the lowest estimated time
        # (pool at the budget's held-out rate + the fixed fraction at the plain rate of the label docking) runs.
        import dataclasses
        import torch
        n_hold = len(sur.holdout_true)
        hold = train.subset(np.arange(args.pf_train - n_hold, args.pf_train))
        hold_dev = P.DeviceLibrary(hold)
        plain_est = args.pf_train / sur.metrics["label_seconds"]
        best = None
        cheap_by_top = {}
        for k in tops:
            cds = P.DeviceSearch(dataclasses.replace(W.search, sweep_top=k, passes=args.pf_cascade_passes))
            P.screen(dp, P.DeviceLibrary(hold.subset(np.arange(min(2000, n_hold)))), cds)  # warm-up
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            cheap_hold = P.screen(dp, hold_dev, cds).best_score.cpu().numpy().astype(np.float64)
            rate = n_hold / (time.perf_counter() - t0)
            cheap_by_top[k] = cheap_hold
            pool = PF.calibrate_cascade(sur.holdout_pred, cheap_hold, sur.holdout_true, fixed,
                                        args.pf_target + args.pf_margin)
            est = args.pf_lib * (pool / rate + fixed / plain_est)
            alone = PF.recall_curve(PF.ranks(cheap_hold), sur.holdout_true, [fixed], n_hold)[fixed]
            candidates.append({"sweep_top": k, "pool_fraction": pool, "held_out_budget_ligands_per_s": rate,
                               "held_out_recall_of_budget_alone": alone, "estimated_seconds": est})
            log(f"cascade candidate: best {k} rigid starts swept, pool {pool:.0%}, held-out budget rate "
                f"{rate:.0f}/s, estimated {est:.1f} s")
            if pool < 1.0 and (best is None or est < best[0]):
                best = (est, k, pool, cds)
        if best is not None:
            _, cascade_top, pool, cascade_ds = best
            pools = (pool,)
            # the same budget with a pool calibrated to a higher held-out recall: what more margin costs
            safe_target = args.pf_target + args.pf_margin + args.pf_cascade_safety
            safe_pool = PF.calibrate_cascade(sur.holdout_pred, cheap_by_top[cascade_top], sur.holdout_true, fixed,
                                             safe_target) if args.pf_cascade_safety > 0 else 1.0
            if pool < safe_pool < 1.0:
                pools = (pool, safe_pool)
                log(f"cascade with more margin: pool {safe_pool:.0%} (held-out target {safe_target:.2f})")
            cascade_how = (f"budget and pool = the fastest estimate among {tops} rigid starts swept, each with the "
                           f"smallest pool reaching held-out cascade recall >= {args.pf_target + args.pf_margin:.2f}")
            log(f"cascade: pool {pool:.0%} docked with the best {cascade_top} rigid starts swept "
                f"({args.pf_cascade_passes} pass), then the top {fixed:.0%} in full")
    res = PF.filtered_screen(sur, dp, ds, W.dist, W.n_types, args.pf_lib, args.pf_chunk, frac,
                             sample_every=args.pf_sample_every, log=log,
                             extra_fracs=(fixed,) if fixed > 0 and abs(fixed - frac) > 1e-9 else (),
                             cascade_search=cascade_ds, cascade_pools=pools, cascade_final=fixed)
    sid, ssc = res["sample_ids"], res["sample_scores"].astype(np.float64)
    recall = PF.recall_top(sid, ssc, res["selected_ids"], 0.01)
    fracs = [0.01, 0.02, 0.03, 0.05, 0.075, 0.1, 0.15, 0.2, 0.3]
    curve = PF.recall_curve(PF.ranks(res["predictions"])[sid], ssc, fracs + [frac], args.pf_lib)
    # the method without the network, at the same budgets: largest ligands first (ties by id), random
    size_rank = PF.ranks(-res["n_atoms"].astype(np.float64))[sid]
    curve_size = PF.recall_curve(size_rank, ssc, fracs + [frac], args.pf_lib)
    small_rank = PF.ranks(res["n_atoms"].astype(np.float64))[sid]
    curve_small = PF.recall_curve(small_rank, ssc, fracs + [frac], args.pf_lib)
    rng = np.random.default_rng(0)
    rand_rank = rng.permutation(args.pf_lib)[sid]
    curve_rand = PF.recall_curve(rand_rank, ssc, fracs + [frac], args.pf_lib)
    n_sample = len(sid)
    plain_rate = n_sample / res["seconds_dock_sample"]
    filtered_seconds = res["seconds_predict"] + res["seconds_dock_selected"]
    out = {
        "metric": "recall@top1% with surrogate; filtered vs plain ligands/s on 1 MI355X",
        "value": recall, "unit": "recall", "higher_is_better": True, "n_gpus": 1, "data": "synthetic",
        "dtype": "bf16 MLP (FP32 accumulation), f32 docking",
        "config": {"workload": f"{W.name}; surrogate trained on {args.pf_train} docked ligands; library of "
                               f"{args.pf_lib} streamed in chunks of {args.pf_chunk}; top {frac:.1%} docked ({how}); "
                               f"recall sample = ids divisible by {args.pf_sample_every} ({n_sample} ligands)"},
        "selected_fraction": frac,
        "target_recall": args.pf_target,
        "surrogate": sur.metrics,
        "filtered_ligands_per_s": args.pf_lib / filtered_seconds,
        # the same with the one-off cost of docking the training ligands and training the networks
        "filtered_ligands_per_s_incl_training": args.pf_lib / (filtered_seconds + sur.metrics["label_seconds"]
                                                               + sur.metrics["train_seconds"]),
        "plain_ligands_per_s": plain_rate,
        "plain_seconds_extrapolated": args.pf_lib / plain_rate,
        "filtered_seconds": filtered_seconds,
        "seconds_predict": res["seconds_predict"],
        "seconds_dock_selected": res["seconds_dock_selected"],
        "speedup": (args.pf_lib / filtered_seconds) / plain_rate,
        "recall_curve": {f"{k:.3f}": v for k, v in curve.items()},
        "recall_curve_largest_first": {f"{k:.3f}": v for k, v in curve_size.items()},
        "recall_curve_smallest_first": {f"{k:.3f}": v for k, v in curve_small.items()},
        "recall_curve_random": {f"{k:.3f}": v for k, v in curve_rand.items()},
        "holdout_ablation": {"ligands": int(len(hy)), "what": "recall of the held-out ligands' true top 1 % when "
                             "the first fraction by each key is kept; linear = least squares on the same 512 "
                             "features and training ligands as the network (host FP64, ridge 1)",
                             "linear_r2": sur.metrics["linear_holdout_r2"],
                             "linear_spearman": sur.metrics["linear_holdout_spearman"],
                             "curves": ablation},
        "host_generation_seconds": res["seconds_generate_on_host"],
        "n_sample": n_sample,
    }
    for f, e in res["extra"].items():
        fs = e["seconds_predict"] + e["seconds_dock_selected"]
        out[f"fixed_fraction_{f:.3f}"] = {
            "selected_fraction": f, "recall": PF.recall_top(sid, ssc, e["selected_ids"], 0.01),
            "filtered_ligands_per_s": args.pf_lib / fs, "speedup": (args.pf_lib / fs) / plain_rate,
            "filtered_seconds": fs, "seconds_dock_selected": e["seconds_dock_selected"],
            "meets_target": PF.recall_top(sid, ssc, e["selected_ids"], 0.01) >= args.pf_target}
    for i, (f, c) in enumerate(res["cascade"].items()):
        cheap_rate = n_sample / res["seconds_dock_sample_cheap"]
        fs = c["seconds_predict"] + c["seconds_dock_pool"] + c["seconds_select_final"] + c["seconds_dock_selected"]
        rec = PF.recall_top(sid, ssc, c["selected_ids"], 0.01)
        # the same cascade without the network: every ligand docked with the smaller budget, the top
        # fraction by those scores docked in full (recall on the sample, time from the two measured rates)
        no_net = PF.recall_curve(PF.ranks(res["sample_cheap_scores"].astype(np.float64)), ssc, [fixed], n_sample)[fixed]
        no_net_s = args.pf_lib / cheap_rate + fixed * args.pf_lib / plain_rate
        if i > 0:  # the same budget with the pool calibrated to the higher held-out target
            out["cascade_more_margin"] = {
                "pool_fraction": f, "held_out_target": args.pf_target + args.pf_margin + args.pf_cascade_safety,
                "recall": rec, "meets_target": rec >= args.pf_target,
                "filtered_ligands_per_s": args.pf_lib / fs, "speedup": (args.pf_lib / fs) / plain_rate,
                "filtered_seconds": fs, "seconds_dock_pool": c["seconds_dock_pool"],
                "seconds_dock_selected": c["seconds_dock_selected"]}
            continue
        out["cascade"] = {
            "what": (f"top {f:.0%} by prediction docked with the best {cascade_top} of "
                     f"{W.search.n_starts} rigid starts swept ({args.pf_cascade_passes} pass); the top {fixed:.0%} "
                     f"of the library by those scores docked in full"),
            "calibration": cascade_how, "candidates": candidates, "sweep_top": cascade_top,
            "pool_fraction": f, "docked_in_full_fraction": fixed,
            "recall": rec, "meets_target": rec >= args.pf_target,
            "filtered_ligands_per_s": args.pf_lib / fs, "speedup": (args.pf_lib / fs) / plain_rate,
            "filtered_seconds": fs, "seconds_predict": c["seconds_predict"],
            "seconds_dock_pool": c["seconds_dock_pool"], "seconds_dock_selected": c["seconds_dock_selected"],
            "budget_ligands_per_s": c["n_pool"] / c["seconds_dock_pool"],
            "without_network": {"recall": no_net, "ligands_per_s": args.pf_lib / no_net_s,
                                "speedup": (args.pf_lib / no_net_s) / plain_rate,
                                "budget_ligands_per_s_on_sample": cheap_rate}}
    print(json.dumps(out), flush=True)


def prefilter_variants(args):
    """Held-out recall of the pre-filter at small docked fractions under training variants: label
    transforms (clipping the bad tail, rank-to-normal, log), ensemble size and learning schedule.
    The labels are the best scores of the same 200k docked training ligands for every variant."""
    import numpy as np
    from scipy.stats import norm

    from paper_2304_09953_amd import inputs as I
    from paper_2304_09953_amd import pipeline as P
    from paper_2304_09953_amd import prefilter as PF
    W = I.workload("pocket96-lib100k")
    dp, ds = P.DevicePocket(W.pockets[0]), P.DeviceSearch(W.search)
    train = I.make_ligands(args.pf_train, W.dist, W.n_types, stream="train")
    log(f"labels: docking {args.pf_train} training ligands")
    y = PF.dock_scores(dp, ds, train).astype(np.float64)
    n_hold = args.pf_train // 5
    n_tr = args.pf_train - n_hold - n_hold // 2
    true = y[-n_hold:]
    fr = [0.01, 0.02, 0.03, 0.05, 0.1]
    clip = lambda q: (lambda v: np.minimum(v, np.percentile(v[:n_tr], q)))  # noqa: E731
    variants = [("base", lambda v: v, 4, 20, 1e-3), ("clip_p50", clip(50), 4, 20, 1e-3),
                ("clip_p25", clip(25), 4, 20, 1e-3), ("clip_p10", clip(10), 4, 20, 1e-3),
                ("rankgauss", lambda v: norm.ppf((PF.ranks(v) + 0.5) / len(v)), 4, 20, 1e-3),
                ("clip_p25_8m", clip(25), 8, 20, 1e-3), ("clip_p25_lr5e-4_40ep", clip(25), 4, 40, 5e-4),
                ("log_shift", lambda v: np.log(v - v.min() + 1.0), 4, 20, 1e-3)]
    rows = []
    for name, f, members, ep, lr in variants:
        sur = PF.train_surrogate(dp, ds, train, labels=f(y).astype(np.float32), n_holdout=n_hold, members=members,
                                 max_epochs=ep, lr=lr)
        curve = PF.recall_curve(PF.ranks(sur.holdout_pred), true, fr, len(true))
        rows.append({"variant": name, "members": members, "max_epochs": ep, "lr": lr,
                     "recall": {f"{k:.2f}": v for k, v in curve.items()}, "best_epochs": sur.metrics["best_epochs"]})
        log(f"{name}: {curve}")
    print(json.dumps({"metric": "held-out recall of the true top 1 % at small docked fractions, by training variant",
                      "unit": "recall", "n_gpus": 1, "data": "synthetic",
                      "config": {"workload": f"{args.pf_train} docked training ligands of {W.name}",
                                 "held_out": n_hold}, "rows": rows}), flush=True)


def batched_bench(args):
    """The multi-pocket workload.  Per pocket the autotuner times the launch candidates on a sample of
    each size bucket and stores the table.  Then the batched path: the library is packed once per
    chunk and screened against all four pockets inside one graph-replayed chunk (host chunk
    preparation and uploads included), keeping every pocket's top-1000 and the best-site ranking.
    For comparison, the same library resident on the device (uploaded and packed once) is screened
    by one persistent dock_screen launch per pocket."""
    import shutil

    import numpy as np
    import torch

    from paper_2304_09953_amd import batching as Bt
    from paper_2304_09953_amd import inputs as I
    from paper_2304_09953_amd import pipeline as P
    W = I.workload("pockets4-lib250k")
    n_lig = args.n_lig or W.n_lig
    k = 1000
    log(f"generating {n_lig} ligands")
    ligs = W.ligands(n_lig=n_lig)
    arch = Bt.arch_name()
    dps = [P.DevicePocket(p) for p in W.pockets]
    searches = [I.search_for(p, W.search) for p in W.pockets]
    tuned, path = {}, None
    for pocket, dp, srch in zip(W.pockets, dps, searches):
        t0 = time.perf_counter()
        table = Bt.autotune(dp, ligs, srch, per_bucket=args.tune_sample)
        path = Bt.save_table(table, arch, pocket.dims, srch.n_steps)
        tuned[f"{pocket.dims[0]}^3"] = {"seconds": time.perf_counter() - t0,
                                        "params": {str(b): [v["starts_per_item"], v["waves_per_block"]]
                                                   for b, v in table.items()}}
        log(f"pocket {pocket.dims}: autotuned in {tuned[f'{pocket.dims[0]}^3']['seconds']:.1f} s")
    if args.tuning_out and path:
        shutil.copy(path, args.tuning_out)
    # batched: one pack per chunk, four pockets per graph replay
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = Bt.screen_sites(dps, searches, ligs, k=k, chunk=args.chunk, tuned=args.launch_params == "tuned",
                          use_graph=True, log=log)
    torch.cuda.synchronize()
    t_batched = time.perf_counter() - t0
    log(f"batched, shared pack: {t_batched:.1f} s, {len(dps) * n_lig / t_batched:.0f} pairs/s")
    # persistent: the device-resident library, one dock_screen launch per pocket (its default launch)
    t0 = time.perf_counter()
    lib = P.DeviceLibrary(ligs)
    torch.cuda.synchronize()
    t_upload = time.perf_counter() - t0
    rows, t_pers, same = [], 0.0, True
    for pi, (pocket, dp, srch) in enumerate(zip(W.pockets, dps, searches)):
        scr = P.Screener(dp, lib, P.DeviceSearch(srch))
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        r = scr.run()
        ts, ti = P.topk(r.best_score, k)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t1
        t_pers += dt
        best = r.best_score.cpu().numpy()
        same &= bool(np.array_equal(best, res.best[pi]))
        rows.append({"pocket": f"{pocket.dims[0]}^3", "persistent_seconds": dt, "persistent_pairs_per_s": n_lig / dt,
                     "docked": int(np.isfinite(best).sum()), "best_score": float(res.top_s[pi][0]),
                     "top1000_last": float(res.top_s[pi][-1]),
                     "top1000_equal": bool(np.array_equal(ligs.ids[ti.cpu().numpy()].astype(np.int32),
                                                          res.top_i[pi]))})
        log(f"pocket {pocket.dims}: one persistent launch {dt:.1f} s, {n_lig / dt:.0f} ligands/s")
    multi = {"best_score": float(res.site_top_s[0]), "top1000_last": float(res.site_top_s[-1]),
             "top1000_by_pocket": {f"{W.pockets[p].dims[0]}^3": int(np.sum(res.site[res.site_top_i] == p))
                                   for p in range(len(dps))}}
    n_pairs = len(dps) * n_lig
    print(json.dumps({"metric": "ligand-pocket pairs docked/s, one pack per chunk for all pockets, graph-replayed",
                      "unit": "pairs/s", "value": n_pairs / t_batched, "n_gpus": 1, "data": "synthetic",
                      "dtype": "f32",
                      "config": {"workload": (W.name if n_lig == W.n_lig else f"first {n_lig} ligands of " + W.name),
                                 "chunk": args.chunk, "k": k, "tune_sample_per_bucket": args.tune_sample,
                                 "launch_params": args.launch_params},
                      "batched_seconds": t_batched,
                      "persistent": {"pairs_per_s": n_pairs / t_pers, "seconds": t_pers,
                                     "library_upload_and_pack_seconds": t_upload,
                                     "what": "device-resident library, one dock_screen launch per pocket + top-k",
                                     "scores_equal_batched": same},
                      "batched_over_persistent": t_pers / t_batched,
                      "autotuning": tuned, "pockets": rows, "best_site_ranking": multi}), flush=True)


def rescore_bench(args):
    """Pose filtering and rescoring after the screen on the first args.n_lig (default 20000)
    ligands of the 100k workload: cost against the screen, poses kept, and how the ranking moves."""
    import numpy as np
    import torch

    from paper_2304_09953_amd import inputs as I
    from paper_2304_09953_amd import pipeline as P
    W = I.workload("pocket96-lib100k")
    n_lig = args.n_lig or 20000
    ligs = W.ligands(n_lig=n_lig)
    dp = P.DevicePocket(W.pockets[0])
    lib = P.DeviceLibrary(ligs)
    ds = P.DeviceSearch(W.search)
    QT = W.search.n_starts
    ev = lambda: torch.cuda.Event(enable_timing=True)  # noqa: E731
    scr = P.Screener(dp, lib, ds, start_scores=True)
    scr.run()
    P.rescore(dp, lib, ds, scr.start_scores.view(n_lig, QT), args.n_keep, args.rmsd_min)
    torch.cuda.synchronize()
    e0, e1, e2 = ev(), ev(), ev()
    e0.record()
    r = scr.run()
    e1.record()
    res = P.rescore(dp, lib, ds, r.start_scores.view(n_lig, QT), args.n_keep, args.rmsd_min)
    e2.record()
    torch.cuda.synchronize()
    dock_s = r.best_score.cpu().numpy().astype(np.float64)
    resc = res.best_rescore.cpu().numpy().astype(np.float64)
    kept = np.isfinite(res.pose_rescore.cpu().numpy()).sum(1)
    ok = np.isfinite(dock_s)
    k = max(1, int(round(0.01 * ok.sum())))
    ids = np.flatnonzero(ok)
    top_d = set(ids[np.lexsort((ids, dock_s[ok]))[:k]].tolist())
    top_r = set(ids[np.lexsort((ids, resc[ok]))[:k]].tolist())
    from scipy.stats import spearmanr
    out = {"metric": "pose filtering + rescoring after the screen", "unit": "ligands/s",
           "value": n_lig / (e1.elapsed_time(e2) * 1e-3),
           "config": {"workload": f"first {n_lig} ligands of {W.name}", "n_keep": args.n_keep,
                      "rmsd_min": args.rmsd_min},
           "screen_ms": e0.elapsed_time(e1), "rescore_ms": e1.elapsed_time(e2),
           "kept_poses_mean": float(kept[ok].mean()), "kept_poses_hist": np.bincount(kept[ok]).tolist(),
           "best_pose_is_docking_best": float(np.mean(res.best_pose.cpu().numpy()[ok] == 0)),
           "spearman_docking_vs_rescore": float(spearmanr(dock_s[ok], resc[ok]).statistic),
           "top1pct_overlap": len(top_d & top_r) / k}
    log(f"rescore: {out['rescore_ms']:.0f} ms after a {out['screen_ms']:.0f} ms screen; "
        f"{out['kept_poses_mean']:.2f} poses kept per ligand")
    print(json.dumps(out), flush=True)


def knob_tuning(args):
    """Bayesian tuning of (Q, T, translation radius, S, passes, sweep_top, restarts), about 4.1e4
    configurations, for the cheapest screen whose top 1 % keeps args.knob_target of the reference
    search's top 1 % on a sample library; compared with random search at the same number of screens
    (five seeds).  The space is too large to screen every configuration."""
    import numpy as np

    from paper_2304_09953_amd import inputs as I
    from paper_2304_09953_amd import knobs as K
    from paper_2304_09953_amd import pipeline as P
    W = I.workload("pocket96-lib100k")
    pocket = W.pockets[0]
    n_lig = args.n_lig or 4000
    ligs = W.ligands(n_lig=n_lig)
    dp = P.DevicePocket(pocket)
    lib = P.DeviceLibrary(ligs)
    obj = K.ScreenObjective(dp, lib, W.search, top_frac=0.01)
    target = args.knob_target
    t0 = time.perf_counter()
    bo = K.optimize(obj, target, n_init=6, n_iter=args.knob_evals - 6, seed=0, log=log)
    t_bo = time.perf_counter() - t0
    rnd = []
    for s in range(5):
        r = K.random_search(obj, target, args.knob_evals, seed=s)
        rnd.append({"seed": s, "best": r["best"], "feasible": int(sum(h["recall"] >= target for h in r["history"]))})
        log(f"random search seed {s}: best {r['best']}")
    costs = [r["best"]["cost"] if r["best"] else None for r in rnd]
    out = {"metric": "knob tuning: cheapest screen keeping the reference top 1 %", "unit": "s per 1M ligands",
           "value": bo["best"]["cost"] if bo["best"] else None,
           "config": {"workload": f"first {n_lig} ligands of {W.name}", "target_recall": target,
                      "reference": "Q256 x T32 (radius 4 A), S256, one pass, every start",
                      "reference_s_per_1M": obj.ref_seconds / n_lig * 1e6, "screens_per_search": args.knob_evals,
                      "space_size": len(K.grid()), "space": {k: list(v) for k, v in K.SPACE.items()}},
           "bayesian": bo["best"], "bayesian_feasible_screens": int(sum(h["recall"] >= target for h in bo["history"])),
           "bayesian_seconds": t_bo, "bayesian_history": bo["history"],
           "random_search": rnd,
           "random_search_mean_best_cost": (float(np.mean([c for c in costs if c is not None]))
                                            if any(c is not None for c in costs) else None),
           "random_search_none_feasible": int(sum(c is None for c in costs))}
    print(json.dumps(out), flush=True)


def budget_curve(args):
    """Speed and quality of the search-budget variants against the full search on the first
    args.n_lig (default 20000) ligands of the 100k workload: ligands/s, and per variant the mean
    and worst score loss against the full search and the share of the full search's top 1 % that
    the variant's own top 1 % keeps."""
    import dataclasses

    import numpy as np
    import torch

    from paper_2304_09953_amd import inputs as I
    from paper_2304_09953_amd import pipeline as P
    W = I.workload("pocket96-lib100k")
    n_lig = args.n_lig or 20000
    ligs = W.ligands(n_lig=n_lig)
    dp = P.DevicePocket(W.pockets[0])
    lib = P.DeviceLibrary(ligs)
    # (sweep_top, passes, torsion restarts per rigid start)
    variants = [(0, 1, 0), (0, 2, 0), (0, 1, 1), (0, 1, 3), (1024, 1, 0), (256, 1, 0), (256, 2, 0), (64, 1, 0),
                (64, 2, 0), (16, 1, 0), (4, 1, 0), (1, 1, 0)]
    rows, ref = [], None
    for top, passes, restarts in variants:
        srch = dataclasses.replace(W.search, sweep_top=top, passes=passes, restarts=restarts,
                                   init_steps=I.restart_steps(restarts, W.search.n_steps) if restarts else None)
        scr = P.Screener(dp, lib, P.DeviceSearch(srch))
        scr.run()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        scr.run()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        best = scr.best_score.cpu().numpy().astype(np.float64)
        poses = int(scr.pose_count.cpu().item())
        if ref is None:
            ref = best
        ok = np.isfinite(ref)
        loss = (best - ref)[ok]
        k = max(1, int(round(0.01 * ok.sum())))
        top_ref = set(np.flatnonzero(ok)[np.lexsort((np.flatnonzero(ok), ref[ok]))[:k]].tolist())
        top_var = set(np.flatnonzero(ok)[np.lexsort((np.flatnonzero(ok), best[ok]))[:k]].tolist())
        rows.append({"sweep_top": top, "passes": passes, "restarts": restarts, "screen_ms": ms,
                     "ligands_per_s": n_lig / (ms * 1e-3),
                     "poses_per_s": poses / (ms * 1e-3), "mean_score_change": float(loss.mean()),
                     "worst_score_change": float(loss.max()), "best_of_full_or_better": float(np.mean(loss <= 1e-4 * np.maximum(1, np.abs(ref[ok])))),
                     "top1pct_overlap_with_full": len(top_ref & top_var) / k})
        log(f"sweep_top={top} passes={passes} restarts={restarts}: {ms:.0f} ms, {n_lig / (ms * 1e-3):.0f} ligands/s, "
            f"mean change {loss.mean():+.3f}, top-1% overlap {len(top_ref & top_var) / k:.3f}")
    print(json.dumps({"metric": "search-budget speed/quality curve", "unit": "ligands/s",
                      "config": {"workload": f"first {n_lig} ligands of {W.name}", "reference": "sweep_top=0, passes=1"},
                      "rows": rows}), flush=True)


def calibrate_peaks(args):
    """Measured peaks of this GPU: non-packed FP32 FMA rate and read bandwidth of a buffer resident
    in the L2 caches (2 MiB, read by every block) and of one resident in the Infinity Cache only
    (64 MiB, larger than all L2s together)."""
    import torch

    from paper_2304_09953_amd import dock
    out = {}
    ev = lambda: torch.cuda.Event(enable_timing=True)  # noqa: E731
    blocks, iters = 8192, 2048
    sink = torch.empty(blocks * 256, dtype=torch.float32, device="cuda")
    dock.calib_fma_f32(blocks, 16, sink)
    torch.cuda.synchronize()
    best = 0.0
    for _ in range(3):
        e0, e1 = ev(), ev()
        e0.record()
        dock.calib_fma_f32(blocks, iters, sink)
        e1.record()
        torch.cuda.synchronize()
        best = max(best, blocks * 256 * iters * 32 / (e0.elapsed_time(e1) * 1e-3))
    out["fma_f32_tflops"] = best / 1e12
    log(f"FMA: {best / 1e12:.1f} TFLOP/s")
    for name, mib, blk, reps in (("l2", 2, 2048, 64), ("mall", 64, 512, 2)):
        if args.calibrate_peaks != "all" and args.calibrate_peaks != name:
            continue
        best = read_peak(mib, blk, reps)
        out[f"{name}_read_tbps"] = best / 1e12
        out[f"{name}_read_bytes_per_launch"] = blk * reps * (mib << 20)
        log(f"{name} ({mib} MiB buffer): {best / 1e12:.2f} TB/s")
    print(json.dumps(out), flush=True)


def read_peak(mib=2, blk=2048, reps=64):
    """Best of three cache-resident reads (one untimed first): each of blk blocks reads the mib MiB
    buffer reps times; bytes/s."""
    import torch

    from paper_2304_09953_amd import dock
    buf = torch.ones(mib << 18, dtype=torch.float32, device="cuda")
    sink = torch.empty(blk * 256, dtype=torch.float32, device="cuda")
    dock.calib_cache_read(buf, 1, blk, sink)
    torch.cuda.synchronize()
    best = 0.0
    for _ in range(3):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        dock.calib_cache_read(buf, reps, blk, sink)
        e1.record()
        torch.cuda.synchronize()
        best = max(best, blk * reps * (mib << 20) / (e0.elapsed_time(e1) * 1e-3))
    return best


def surrogate_roofline(args):
    """MFMA throughput of the pre-filter network: the forward pass at the prediction chunk size and
    at a large batch, and one training step (forward, backward, Adam) at the training batch, each
    timed with HIP events (best of three after a warm-up) against the dense BF16 peak."""
    import numpy as np
    import torch

    from paper_2304_09953_amd import inputs as I
    from paper_2304_09953_amd import surrogate as SG
    peak = 2.5e15
    d_in, h1, h2 = 512, 1024, 1024
    model = SG.Model(I.mlp_init(d_in, h1, h2))
    fwd_flop = 2.0 * (d_in * h1 + h1 * h2 + h2)  # per row
    gen = torch.Generator(device="cuda").manual_seed(5)
    ev = lambda: torch.cuda.Event(enable_timing=True)  # noqa: E731

    def best_of(fn, reps=3):
        fn()
        torch.cuda.synchronize()
        best = float("inf")
        for _ in range(reps):
            e0, e1 = ev(), ev()
            e0.record()
            fn()
            e1.record()
            torch.cuda.synchronize()
            best = min(best, e0.elapsed_time(e1) * 1e-3)
        return best

    rows = []
    for batch in (65536, 1 << 20):
        x = (torch.randn((batch, d_in), generator=gen, device="cuda") * 0.5).to(torch.bfloat16).view(torch.int16)
        y = torch.empty(batch, dtype=torch.float32, device="cuda")
        t = best_of(lambda: model.forward(x, y))
        rows.append({"pass": "forward", "batch": batch, "seconds": t, "tflops": fwd_flop * batch / t / 1e12,
                     "frac": fwd_flop * batch / t / peak})
        log(f"forward batch {batch}: {t * 1e3:.2f} ms, {fwd_flop * batch / t / 1e12:.1f} TFLOP/s")
        del x, y
    batch = 1024
    x = (torch.randn((batch, d_in), generator=gen, device="cuda") * 0.5).to(torch.bfloat16).view(torch.int16)
    tgt = torch.randn(batch, generator=gen, device="cuda")
    loss = torch.empty(1, dtype=torch.float32, device="cuda")

    def step():
        model.backward(x, tgt, loss)
        model.adam(1e-4)
    t = best_of(step)
    # forward, then the weight and input gradients of the two hidden layers (the input layer needs no
    # input gradient): 3 x forward minus one d_in x h1 product
    step_flop = batch * (3 * fwd_flop - 2.0 * d_in * h1)
    rows.append({"pass": "training step", "batch": batch, "seconds": t, "tflops": step_flop / t / 1e12,
                 "frac": step_flop / t / peak})
    log(f"training step batch {batch}: {t * 1e3:.3f} ms, {step_flop / t / 1e12:.1f} TFLOP/s")
    # reference point: the library BF16 GEMM behind torch.matmul on the first layer's product
    # (no bias, no activation) at the large batch
    xa = torch.randn((1 << 20, d_in), generator=gen, device="cuda").to(torch.bfloat16)
    wa = torch.randn((h1, d_in), generator=gen, device="cuda").to(torch.bfloat16)
    out = torch.empty((1 << 20, h1), dtype=torch.bfloat16, device="cuda")
    t = best_of(lambda: torch.matmul(xa, wa.t(), out=out))
    lib_flop = 2.0 * (1 << 20) * d_in * h1
    rows.append({"pass": "library GEMM (torch.matmul, first layer product only)", "batch": 1 << 20, "seconds": t,
                 "tflops": lib_flop / t / 1e12, "frac": lib_flop / t / peak})
    log(f"torch.matmul {1 << 20} x {d_in} x {h1}: {t * 1e3:.2f} ms, {lib_flop / t / 1e12:.1f} TFLOP/s")
    print(json.dumps({"metric": "pre-filter network MFMA throughput", "unit": "TFLOP/s",
                      "peak": {"bf16_dense_tflops": peak / 1e12},
                      "config": {"network": f"{d_in}-{h1}-{h2}-1, BF16 weights and activations, FP32 accumulation"},
                      "rows": rows}), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n-lig", type=int, default=None, help="dock only the first N ligands (a subset workload)")
    ap.add_argument("--cpu-seconds", type=float, default=12.0, help="time budget of the CPU oracle baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--summarize-counters", metavar="DIR", default=None,
                    help="write the screen's counter summary from rocprofv3 --pmc CSV directories in DIR")
    ap.add_argument("--calibrate-peaks", choices=("all", "l2", "mall", "fma"), default=None,
                    help="measure the FMA rate and cache-resident read bandwidth of this GPU, then exit")
    ap.add_argument("--tune-knobs", action="store_true",
                    help="Bayesian tuning of the search knobs on --n-lig ligands (default 4000)")
    ap.add_argument("--knob-target", type=float, default=0.9, help="recall of the reference top 1 %% to keep")
    ap.add_argument("--knob-evals", type=int, default=40, help="screens per tuning search")
    ap.add_argument("--rescore", action="store_true",
                    help="pose filtering and rescoring after the screen on --n-lig ligands (default 20000)")
    ap.add_argument("--n-keep", type=int, default=8, help="poses kept per ligand before filtering (--rescore)")
    ap.add_argument("--rmsd-min", type=float, default=1.0, help="RMSD (Angstrom) below which a pose is dropped")
    ap.add_argument("--batched", action="store_true",
                    help="the 4-pocket workload through the autotuned, graph-replayed batching path")
    ap.add_argument("--chunk", type=int, default=16384, help="ligands per graph-replayed chunk (--batched)")
    ap.add_argument("--tune-sample", type=int, default=2048, help="ligands per size bucket timed by the autotuner")
    ap.add_argument("--tuning-out", default=None, help="also copy the autotuner table here (--batched)")
    ap.add_argument("--launch-params", choices=("tuned", "library"), default="tuned",
                    help="--batched: chunks use the autotuned launch parameters, or the library's own choice")
    ap.add_argument("--budget-curve", action="store_true",
                    help="speed and quality of the search-budget variants (sweep_top, passes) against the full "
                         "search on --n-lig ligands (default 20000)")
    ap.add_argument("--layout", choices=("xy4", "linear"), default="xy4",
                    help="grid layout: 16-byte records of the four xy neighbours, or plain [t][z][y][x]")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (reference for the HBM byte counters)")
    ap.add_argument("--prefilter", action="store_true",
                    help="measure the learned pre-filter instead: train on docked labels, filter a streamed "
                         "library, dock the selection, recall of the true top 1%% of a fully docked sample")
    ap.add_argument("--pf-train", type=int, default=200_000)
    ap.add_argument("--prefilter-variants", action="store_true",
                    help="held-out recall of pre-filter training variants at small docked fractions")
    ap.add_argument("--pf-lib", type=int, default=10_000_000)
    ap.add_argument("--pf-chunk", type=int, default=1_000_000)
    ap.add_argument("--pf-sample-every", type=int, default=20, help="recall sample: ids divisible by this")
    ap.add_argument("--pf-fixed-frac", type=float, default=0.03,
                    help="also dock this fixed top fraction from the same predictions (0: skip)")
    ap.add_argument("--pf-frac", type=float, default=0.0,
                    help="fraction docked after the filter; 0 = calibrated on the held-out docked ligands")
    ap.add_argument("--pf-target", type=float, default=0.95, help="recall of the true top 1%% to reach")
    ap.add_argument("--pf-margin", type=float, default=0.02, help="added to the target when calibrating")
    ap.add_argument("--pf-epochs", type=int, default=20, help="most epochs per member (early stopping)")
    ap.add_argument("--pf-members", type=int, default=4, help="networks in the ensemble")
    ap.add_argument("--pf-cascade-tops", default="256,512,1024,2048",
                    help="cascade: candidate numbers of rigid starts swept in the pool's budgeted docking, "
                         "comma-separated ('' = no cascade)")
    ap.add_argument("--pf-cascade-passes", type=int, default=1, help="cascade: greedy passes of the budgeted docking")
    ap.add_argument("--pf-cascade-safety", type=float, default=0.01,
                    help="cascade: also dock a pool calibrated to this much more held-out recall (0: no)")
    ap.add_argument("--surrogate-roofline", action="store_true",
                    help="MFMA throughput of the pre-filter network's forward pass and training step")
    args = ap.parse_args()
    if args.summarize_counters:
        return summarize_counters(args.summarize_counters)
    if args.gpus != 1:
        print("bench.py measures one GPU only: the screen has no multi-GPU path (a library would be sharded "
              "by ligand over independent processes). Use --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2304_09953_amd import dock
    from paper_2304_09953_amd import inputs as I
    from paper_2304_09953_amd import pipeline as P

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.calibrate_copy:
        n = args.calibrate_copy * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": 4 * n, "launches": 1}), flush=True)
        return
    dock.load()  # fails loudly if the HIP library is missing
    if args.calibrate_peaks:
        return calibrate_peaks(args)
    if args.budget_curve:
        return budget_curve(args)
    if args.batched:
        return batched_bench(args)
    if args.rescore:
        return rescore_bench(args)
    if args.tune_knobs:
        return knob_tuning(args)
    if args.prefilter_variants:
        return prefilter_variants(args)
    if args.prefilter:
        return prefilter_bench(args)
    if args.surrogate_roofline:
        return surrogate_roofline(args)
    W = I.workload("pocket96-lib100k")
    n_lig = args.n_lig or W.n_lig
    log(f"generating {n_lig} ligands")
    ligs = W.ligands(n_lig=n_lig)
    pocket = W.pockets[0]
    S, QT, K_TOP = W.search.n_steps, W.search.n_starts, 1000

    layout = dock.LAYOUT_XY4 if args.layout == "xy4" else dock.LAYOUT_LINEAR
    dp = P.DevicePocket(pocket, layout=layout)
    torch.cuda.synchronize()
    t_up = time.perf_counter()
    lib = P.DeviceLibrary(ligs)  # host CSR arrays -> device (allocation included)
    torch.cuda.synchronize()
    upload_s = time.perf_counter() - t_up
    ds = P.DeviceSearch(W.search)
    scr = P.Screener(dp, lib, ds)
    k = min(K_TOP, n_lig)
    topk_ws = torch.empty(dock.topk_ws_bytes(n_lig, k), dtype=torch.uint8, device="cuda")
    top_s = torch.empty(k, dtype=torch.float32, device="cuda")
    top_i = torch.empty(k, dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()

    ev = []

    def step():
        dock.build_grids(dp.desc, dp.prot_xyz, dp.prot_type, pocket.type_R, pocket.type_eps, pocket.type_q,
                         pocket.cap, pocket.r_min, pocket.coulomb_k, dp.grids)
        dock.pack_ligands(lib.atom_off, lib.xyz, lib.types, lib.bond_off, lib.bonds, lib.rot, lib.n_types, lib.pack,
                          lib.status)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        scr.run()
        e1.record()
        dock.topk(scr.best_score, k, top_s, top_i, topk_ws)
        ev.append((e0, e1))

    for i in range(args.warmup):
        step()
        torch.cuda.synchronize()
        log(f"warmup step {i + 1}/{args.warmup} done")
    ev.clear()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step()
        torch.cuda.synchronize()
        log(f"timed step {i + 1}/{args.steps} done ({time.perf_counter() - t0:.2f} s)")
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    screen_ms = float(np.mean([a.elapsed_time(b) for a, b in ev]))

    desc = lib.descriptors()
    ok = desc["status"] == 0
    n_at, B, sum_m = desc["n"][ok].astype(np.int64), desc["B"][ok].astype(np.int64), desc["sum_m"][ok].astype(np.int64)
    poses = int(np.sum(QT * (1 + B * (S - 1))))
    assert poses == int(scr.pose_count.cpu().item())
    # a sweep of torsion k looks up its moving atoms but its axis atom b: b lies on the axis, so its grid
    # term does not change with the angle and is not needed (|M_k| - 1 lookups per step)
    swept = sum_m - B
    lookups = int(np.sum(QT * (n_at + (S - 1) * swept)))
    lookups_with_axis = int(np.sum(QT * (n_at + (S - 1) * sum_m)))
    flop = int(np.sum(QT * (FLOP_RIGID_ATOM * n_at + FLOP_SWEEP_LOOKUP * (S - 1) * swept)))
    flop_kernel = int(np.sum(QT * (FLOP_RIGID_ATOM_KERNEL * n_at + FLOP_SWEEP_LOOKUP_KERNEL * (S - 1) * swept)))
    achieved = flop / (screen_ms * 1e-3)
    best = scr.best_score.cpu().numpy()
    assert np.all(np.isfinite(best[ok]))
    t_screen = screen_ms * 1e-3
    c = counters() if n_lig == W.n_lig else None  # the counters are per launch of the full workload
    l2_peak = read_peak()
    log(f"L2-resident read peak: {l2_peak / 1e12:.2f} TB/s")
    gather = {
        "algorithmic_bytes_per_s": BYTES_PER_LOOKUP * lookups / t_screen,
        "l1_to_l2_bytes_per_s": c["l1_to_l2_bytes_per_launch"] / t_screen if c else None,
        "l2_read_peak_bytes_per_s": l2_peak,
        "frac": c["l1_to_l2_bytes_per_launch"] / t_screen / l2_peak if c else None,
        "algorithmic_frac": BYTES_PER_LOOKUP * lookups / t_screen / l2_peak,
        "l2_hit_rate": c["l2_hit_rate"] if c else None,
        "l1_to_l2_requests_per_lookup": c["l1_to_l2_requests_per_launch"] / lookups if c else None,
        "l2_misses_per_lookup": c["l2_misses_per_launch"] / lookups if c and "l2_misses_per_launch" in c else None,
        "hbm_side_bytes_per_s": c["hbm_bytes_per_launch"] / t_screen if c else None,
        "hbm_side_frac": c["hbm_bytes_per_launch"] / t_screen / 8e12 if c else None,
        "valu_busy": c["valu_busy"] if c else None,
        "note": "frac: L1-to-L2 request bytes (rocprofv3, per launch) over the measured L2-resident read peak; "
                "algorithmic_frac: the lookups' 32 B each over the same peak (the bytes the lanes gather, "
                "L1 hits included); HBM side = FETCH_SIZE + WRITE_SIZE (Infinity Cache hits included) "
                "over 8 TB/s",
    }

    out = {
        "metric": METRIC,
        "value": n_lig * args.steps / dt,
        "unit": "ligands/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * dt / args.steps,
        # the C ABI takes device buffers; for reference, the rate with the library's host-to-device
        # upload added to each step (never the headline value)
        "library_upload_ms": 1e3 * upload_s,
        "upload_inclusive_ligands_per_s": n_lig / (dt / args.steps + upload_s),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": (W.name if n_lig == W.n_lig else f"first {n_lig} ligands of " + W.name)
                   + "; top-1000",
                   "n_lig": n_lig, "grid": "96^3x16", "grid_layout": args.layout, "search": "Q256xT32xS256",
                   "top_k": k, "seed": I.BASE_SEED},
        "poses_per_sec": poses * args.steps / dt,
        "screen_ms": screen_ms,
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP32_NONPACKED / 1e12,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_NONPACKED, "traffic": traffic_from_counters(),
                     "kernel": "k_screen (+ its planning and replay kernels, inside the same events)",
                     "algorithmic_flop_per_launch": flop, "lookups_per_launch": lookups,
                     "lookups_per_launch_counting_axis_atoms": lookups_with_axis,
                     "flop_units": {"rigid_atom": FLOP_RIGID_ATOM, "sweep_lookup": FLOP_SWEEP_LOOKUP},
                     "kernel_count_units": {"rigid_atom": FLOP_RIGID_ATOM_KERNEL,
                                            "sweep_lookup": FLOP_SWEEP_LOOKUP_KERNEL,
                                            "achieved": flop_kernel / (screen_ms * 1e-3) / 1e12,
                                            "frac": flop_kernel / (screen_ms * 1e-3) / PEAK_FP32_NONPACKED},
                     "gather_bytes_per_s": BYTES_PER_LOOKUP * lookups / (screen_ms * 1e-3)},
        "gather_roofline": gather,
        # the paper's only throughput figure, as context (not comparable: its ligands, sites, search
        # and scoring differ, and the machines are not named)
        "paper_context": {"ligands_per_s": 7e10 / (60 * 3600.0),
                          "what": "campaign total: more than 7e10 ligands against 15 sites in 60 h (paper, section 2)",
                          "hardware": "two supercomputers, 81 PFLOP/s combined peak, machines and precision not stated"},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(W, ligs, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
