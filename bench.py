#!/usr/bin/env python3
"""Throughput of one step of the CSE hot path on one MI355X.

Default workload (the metric's configuration): 2-arm binomial design (n = 35 per arm, pooled
two-proportion z, reject z > 1.96), all 1024 x 1024 boxes on logit [-3, 1]^2 (2^20 tiles, of them
524,800 meeting the null theta1 <= theta0, 1,024 cut into triangles), 16,384 simulations per tile,
seed 0, alpha 2.5%, delta 1%.  --workload selects the others (listed in WORKLOADS); the default run
also measures the 256 x 256 calibration grid and the 4-arm hierarchical calibration as sub-records.

One step = one call of cse_calibrate with every output requested: the inverted Tilt-Bound
target alpha'_i and k_i, the fused simulation (Philox common random numbers, draws, design
statistic, rejection counts at the fixed cut, score sums for the gradient, per-simulation
calibration records), the order-statistic selection lambda*_i and its count below,
lambda* = min over the tiles in the null space, the gradient, and the Clopper-Pearson +
Tilt-Bound of every tile.  The basket workload is validation only.  The platten (null clipping,
vertices, thresholds, batch plan, 4-arm posterior table) is built once before timing and
reported separately.

The oracle baseline runs first, before anything touches the GPU: the C/numpy oracle on a
bounded uniform sample of the same workload, on one core and then on all cores this process may
use (at most 16, by fork), with the CPU model and core counts stated.

Prints one JSON line.  --gpus above 1 is refused: the library runs on one GPU.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "sim·tiles/s, TIE+gradient+calibration vs plain fwd at equal bound; % roofline"
VALU_PEAK = 256 * 4 * 64 * 2.4e9 / 4   # lane-ops/s: 256 CUs x 4 SIMDs x one wave64 op per 4 clocks

# Algorithmic integer work per unit (lane-ops), by fused kernel:
#   2-arm: per (workgroup, simulation) 18 Philox blocks x 10 rounds x (2 32x32->64 products
#   + 2 xor3), shared by the 16 batches of the group's 4 x 4 square, and the square's 8 sets of
#   8 thresholds x 35 words x (compare + add), each counted once; per (simulation, tile) decision
#   (med3), packed multiply-add and its share of the count unpacking (the calibration record is
#   one 16-byte store per (simulation, batch)).
B2_PHILOX, B2_COUNT_G, B2_TILE_CAL, B2_TILE_FWD = 18 * 10 * 4, 8 * 8 * 35 * 2, 4, 4
#   4-arm: per (workgroup, simulation) 35 Philox blocks; per (batch, simulation) 35 words x
#   (4 + 4 + 2 + 2) thresholds x (compare + add); per (simulation, box) outcome index (3),
#   table gather (1), 3 compares, mask, 2 accumulates; per (simulation, tile) min + key store
#   (the score sums add per rejecting simulation only, a few % of the simulations).
H4_PHILOX, H4_COUNT, H4_BOX, H4_TILE = 35 * 10 * 4, 35 * 12 * 2, 9, 3
#   basket (the same kernel, one configuration per slot): per (simulation, piece) outcome index
#   (3), table gather (1), 4 compares, mask, event test, accumulate.
BK_SLOT = 11

#   Phase II/III: float64 lane-ops of one posterior look (hier_post.hpp), counted by operation
#   (exp 20, log 30, log1p series 22, erfc 40, reciprocal 5, sqrt 10; the per-node constants
#   come from a table): per node 400 outside Newton and the normal tails, 200 per Newton step,
#   104 per arm whose tails a look needs (two erfc); per Phase II look p_best 6,500 + p_success
#   300 (no tails); per Phase III look one p_success (100) and the selected arm's tails.  The
#   first look of a trial is a table lookup (no posterior).  Looks and Newton steps are the
#   kernel's own counters for the launch (cse_work_counters).
P23_NODE, P23_NEWTON, P23_TAIL, P23_P2_EXTRA, P23_P3_EXTRA = 400, 200, 104, 6800, 100

# HBM bytes per dispatch of the dominant kernel, by workload, from FETCH_SIZE + WRITE_SIZE counter
# runs (profiles/<workload>_counters.md, scaled by what the counters read for a copy of known
# size).  Valid only while that kernel is unchanged; workloads not listed report null.
TRAFFIC = {
    "binom2_1024_full": 4_388_248_490,   # k_binom2<true>: 17.8 MB read, 4,370.5 MB written (records + sums)
    "hier4_16": 11_977_047_296,          # k_hier4<1, false, true>: 3,567.7 MB read, 8,409.3 MB written
    "phase23_c5_sub256": 1_625_325_749,  # k_phase23: 228.7 MB read, 1,396.7 MB written
}

DEFAULT = "binom2_1024_full"
SUB_RECORDS = ("binom2_256_tri", "hier4_16")


def b2_method_min_ops(P, w, calibrating):
    """The 2-arm method's own integer work per launch, each distinct threshold counted once per
    simulation: per (N class, simulation) 18 Philox blocks and 35 compare-adds at every distinct
    arm-0 and arm-1 threshold of the class, plus the per-(simulation, tile) decision and accumulate
    (and record share) -- the count that batching can approach but not go below."""
    import numpy as np

    th = np.asarray(P.tiles["theta"])
    sims = np.asarray(w["sims"])[np.asarray(P.tiles["box"])]
    total = 0
    for N in np.unique(sims):
        sel = sims == N
        u = len(np.unique(th[sel, 0])) + len(np.unique(th[sel, 1]))
        total += int(N) * (B2_PHILOX + u * 35 * 2) + int(N) * int(sel.sum()) * (B2_TILE_CAL if calibrating
                                                                                else B2_TILE_FWD)
    return total

WORKLOADS = {
    "binom2_256_tri": "binom2 n=35 pooled-z, 256x256 boxes on [-3,1]^2 kept to theta1<=theta0 "
                      "(32,896 tiles), 8,192 sims/tile, seed 0, alpha 0.025, delta 0.01; "
                      "step = calibrate + validate + gradient",
    "binom2_1024_full": "binom2 n=35 pooled-z, all 1024x1024 boxes on [-3,1]^2 (1,048,576 tiles simulated, "
                        "524,800 meet theta1<=theta0), 16,384 sims/tile, seed 0, alpha 0.025, delta 0.01; "
                        "step = calibrate (lambda* over the null tiles) + validate + score gradient",
    "hier4_16": "hier4 n=35 hierarchical Bayes (90-node sigma^2 quadrature), 16^4 boxes on [-1,1]^4 clipped "
                "to the null configurations, 32,768 sims/tile, seed 0, alpha 0.025, delta 0.01; "
                "step = calibrate + validate",
    "ztest1d_64": "1-D z-test, 64 tiles on [-1,0], 10,000 sims/tile, seed 0, alpha 0.025, delta 0.01; "
                  "step = calibrate + validate + gradient",
    "phase23_c5": "Phase II/III selection design (350/arm embedding, hierarchical posterior at every look), "
                  "16x16x32x32 boxes on logit [-0.9946,1.1527]^4 clipped to the null configurations, "
                  "2^(11+g) sims per box (g uniform on 0..5, PCG64(0)), seed 0, lambda 0.06253, alpha 0.025, "
                  "delta 0.01; step = calibrate + validate + gradient",
    "phase23_c5_sub256": "the Phase II/III workload restricted to every 256th box (1,024 boxes), same sims "
                         "per box; step = calibrate + validate + gradient",
    "basket4_16": "Bayesian basket design (4 arms, n=35, 85% posterior rule, hierarchical model on the "
                  "offsets from p_0a = 15% assumed for every arm), 16^4 boxes on [-3.5,1]^4 cut at the null "
                  "boundaries into pieces (73,521 tiles), 32,768 sims per piece, seed 0, delta 0.01; "
                  "step = validate (rejections at the 85% rule + Clopper-Pearson + Tilt-Bound)",
    "binom2_adaptive": "binom2 n=35 pooled-z on [-3,1]^2 kept to theta1<=theta0, adaptive validation from "
                       "16x16 boxes with 2,048 sims: rounds of GPU validation of the changed boxes, then split "
                       "(half-width down to 1/128, the 256x256 grid's) or double N (up to 131,072) where the "
                       "bound exceeds 0.03; seed 0, delta 0.01, at most 12 rounds; step = the whole adaptive run",
}

ADAPTIVE = dict(target=0.03, delta=0.01, r_min=1.0 / 128, n_max=1 << 17, max_rounds=12)


def run_adaptive(args):
    """The adaptive-gridding workload: a step is one whole adaptive run (every round's GPU
    validation of the changed boxes, the library's host decisions, platten builds)."""
    import numpy as np
    import torch

    import paper_2212_10042_amd as cse
    import paper_2212_10042_amd.adagrid as AG
    import workloads as W

    w = W.binom2_grid(16, 2048, seed=0)

    def once(progress=False):
        return AG.run("binom2", w["theta"], w["radii"], w["sims"], seed=0, mode="validate", **ADAPTIVE,
                      on_round=(lambda r, h: print(f"bench.py: round {r}: boxes, splits, doubles, stuck, "
                                                   f"sims = {h}", file=sys.stderr, flush=True))
                      if progress else None)

    for _ in range(args.warmup):
        once()
    torch.cuda.synchronize()
    cse.cse_profile_reset()
    cse.cse_profile_enable(True)
    t = time.perf_counter()
    for i in range(args.steps):
        res = once(progress=args.progress and i == 0)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t) / args.steps
    cse.cse_profile_enable(False)
    kern = {}
    for kn in ("binom2", "bound_validate"):
        cnt, ms = cse.cse_profile_get(kn)
        if cnt:
            kern[kn] = {"launches_per_step": cnt // args.steps, "ms_per_step": ms / args.steps}
    spent = sum(h[4] for h in res["history"])
    # the same domain on a uniform grid at the finest half-width, with the largest N used
    m = int(round(4.0 / (2 * ADAPTIVE["r_min"])))
    uniform = (m * (m + 1) // 2) * int(res["sims"].max())
    U = np.full(len(res["sims"]), -np.inf)
    np.maximum.at(U, res["tile_box"], res["a"])
    cpu = None
    if not args.no_cpu_baseline:
        import oracle as O
        rng = np.random.default_rng(1234)
        idx = np.sort(rng.choice(len(res["sims"]), min(len(res["sims"]), 24), replace=False))
        tt = time.perf_counter()
        v = O.validate("binom2", res["theta"][idx], res["radii"][idx], res["sims"][idx], 0, ADAPTIVE["delta"])
        dtc = time.perf_counter() - tt
        st = int(res["sims"][idx][np.unique(v["box"])].sum())
        cpu = {"value": st / dtc, "unit": "sim·tiles/s", "cores": 1, "kind": "oracle",
               "sample": f"oracle validate of {len(idx)} of the final boxes (uniform, seed 1234) at their final "
                         f"sims, {dtc:.1f} s single-threaded"}
    out = {
        "metric": METRIC, "value": spent / dt, "unit": "sim·tiles/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": dt * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u32/f32/f64", "data": "synthetic",
        "config": {"workload": WORKLOADS["binom2_adaptive"], "name": "binom2_adaptive",
                   "parallelism": "single GPU"},
        "adaptive": {"rounds": res["rounds"], "history": [list(h) for h in res["history"]],
                     "final_boxes": len(res["sims"]), "final_tiles": len(res["tile_box"]),
                     "sims_simulated": spent, "uniform_equivalent_sims": uniform,
                     "savings": uniform / spent, "max_final_bound": float(U.max()),
                     "boxes_above_target": int(np.sum(U > ADAPTIVE["target"])),
                     "stuck_boxes": int(np.sum(res["decision"] == 3)),
                     "sims_range": [int(res["sims"].min()), int(res["sims"].max())],
                     "half_width_range": [float(res["radii"].min()), float(res["radii"].max())]},
        "kernel_per_step": kern,
        "roofline": None,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_run(args):
    """One oracle pass (validate, and calibrate where the GPU step calibrates) over sampled boxes;
    returns (seconds, sim-tiles)."""
    import numpy as np

    import oracle as O
    import workloads as W

    name, w, design, idx = args
    keep_all = name == "binom2_1024_full"
    validation_only = name == "basket4_16"
    cut = w.get("cut", 0.05 if design == "hier4" else 1.96)
    s = W.subsample(w, idx)
    if design == "phase23":
        s["sims"] = np.minimum(s["sims"], 256).astype(np.int32)   # ~0.6 ms per oracle trial
    t = time.perf_counter()
    v = O.validate(design, s["theta"], s["radii"], s["sims"], w["seed"], w["delta"], cut=cut, keep_all=keep_all)
    if not validation_only:
        O.calibrate(design, s["theta"], s["radii"], s["sims"], w["seed"], w["alpha"], cut=cut, keep_all=keep_all,
                    key_dtype=np.float32 if design in ("hier4", "phase23") else np.float64)
    return time.perf_counter() - t, int(np.asarray(s["sims"])[v["box"]].sum()), len(v["box"])


def cpu_baseline(name, w, design, target_s: float = 8.0, par_target_s: float = 3.0):
    """The oracle as it stands, same step as the GPU, on uniform samples of boxes of the same
    workload: one core, then all usable cores (at most 16) each taking a share of a larger sample.
    Runs before the GPU is initialised, so the worker processes are forked safely."""
    import multiprocessing as mp

    import numpy as np

    rng = np.random.default_rng(1234)
    n = w["theta"].shape[0]
    dt, _, _ = _oracle_run((name, w, design, np.sort(rng.choice(n, 4, replace=False))))
    per_box = max(dt, 1e-3) / 4
    m1 = int(min(n, max(4, target_s / per_box)))
    idx1 = np.sort(rng.choice(n, m1, replace=False))
    dt1, st1, nt1 = _oracle_run((name, w, design, idx1))
    cores = max(1, min(16, len(os.sched_getaffinity(0))))
    mp_ = int(min(n, max(cores, cores * par_target_s / per_box)))
    idxp = np.sort(rng.choice(n, mp_, replace=False))
    parts = [(name, w, design, idxp[i::cores]) for i in range(cores)]
    t = time.perf_counter()
    with mp.get_context("fork").Pool(cores) as pool:
        res = pool.map(_oracle_run, parts)
    dtp = time.perf_counter() - t
    stp = sum(r[1] for r in res)
    ntp = sum(r[2] for r in res)
    sims_note = "min(N, 256) sims of each" if design == "phase23" else "all sims of each"
    step = "validate" if name == "basket4_16" else "validate + calibrate"
    return {"value": stp / dtp, "unit": "sim·tiles/s", "cores": cores, "kind": "oracle",
            "sample": f"{mp_} boxes ({ntp} tiles) drawn uniformly (seed 1234) of the same workload, {sims_note}, "
                      f"split over {cores} forked processes: oracle {step}, {dtp:.1f} s wall",
            "one_core": {"value": st1 / dt1, "cores": 1,
                         "sample": f"{m1} boxes ({nt1} tiles), {sims_note}: oracle {step}, {dt1:.1f} s"},
            "cpu_model": _cpu_model(), "nproc": os.cpu_count(), "usable_cores": len(os.sched_getaffinity(0))}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", choices=sorted(WORKLOADS), default=DEFAULT)
    ap.add_argument("--no-sub", action="store_true", help="skip the sub-record workloads of the default run")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--autotune", action="store_true",
                    help="pick the fused kernel's launch shape with cse_autotune before timing")
    ap.add_argument("--no-graph", action="store_true", help="skip the HIP-graph replay measurement")
    ap.add_argument("--b2-margin", type=float, default=None,
                    help="2-arm calibration: the selection's bracket margin in standard deviations (default 5)")
    ap.add_argument("--h4-bracket", action="store_true",
                    help="4-arm calibration from bracketed keys (pilot + in-bracket candidates) instead of every key")
    ap.add_argument("--no-extensions", action="store_true",
                    help="skip the lower-bound, confidence-set and randomised-calibration timings")
    ap.add_argument("--progress", action="store_true",
                    help="synchronise and report on stderr after every step (for steps of a minute or more)")
    ap.add_argument("--copy-probe", type=int, default=0,
                    help="only copy this many bytes device-to-device 3 times (scales HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: one GPU only (--gpus 1); multi-GPU sharding is not implemented",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np

    import workloads as W

    if args.workload == "binom2_adaptive":
        import torch
        torch.cuda.set_device(0)
        run_adaptive(args)
        return
    if args.copy_probe:
        import torch
        torch.cuda.set_device(0)
        src = torch.ones(args.copy_probe // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": args.copy_probe, "copies": 3}), flush=True)
        return
    name = args.workload
    w, design = load_workload(name)
    # the oracle first: its worker processes are forked before anything initialises the GPU
    cpu = None if args.no_cpu_baseline else cpu_baseline(name, w, design)
    import torch
    torch.cuda.set_device(0)
    res = measure(name, w, design, args, full=True)
    res["cpu_baseline"] = cpu
    if name == DEFAULT and not args.no_sub:
        res["sub_records"] = {}
        for sub in SUB_RECORDS:
            ws, ds = load_workload(sub)
            r = measure(sub, ws, ds, args, full=False)
            res["sub_records"][sub] = {k: r[k] for k in ("value", "unit", "ms_per_step", "steps", "config",
                                                        "kernel_avg_ms", "roofline", "speedup_vs_plain_fwd",
                                                        "lambda_global") if k in r}
    print(json.dumps(res), flush=True)


def load_workload(name):
    import numpy as np

    import workloads as W

    if name == "phase23_c5_sub256":
        w5 = W.phase23_c5()
        w = W.subsample(w5, np.arange(0, w5["theta"].shape[0], 256))
    else:
        w = getattr(W, name)()
    design = {"binom2_256_tri": "binom2", "binom2_1024_full": "binom2", "hier4_16": "hier4",
              "ztest1d_64": "ztest1", "phase23_c5": "phase23", "phase23_c5_sub256": "phase23",
              "basket4_16": "basket4"}[name]
    return w, design


def measure(name, w, design, args, full=True):
    """Time `args.steps` steps of workload `name` after `args.warmup`; with full=False (sub-records)
    at most 10 steps and no graph, extension or Taylor timings."""
    import numpy as np
    import torch

    import paper_2212_10042_amd as cse

    steps = args.steps if full else min(args.steps, 10)
    warmup = args.warmup if full else min(args.warmup, 2)
    keep_all = name == "binom2_1024_full"
    calibrating = name != "basket4_16"
    t0 = time.perf_counter()
    P = cse.Platten.create(design, w["theta"], w["radii"], w["sims"], keep_all=keep_all, cut=w.get("cut"))
    platten_ms = (time.perf_counter() - t0) * 1e3
    if args.h4_bracket and design == "hier4":
        cse.cse_platten_set_option(P.handle, cse.CSE_OPT_H4_BRACKET, 1)
    if args.b2_margin is not None and design == "binom2":
        cse.cse_platten_set_option(P.handle, cse.CSE_OPT_B2_MARGIN, args.b2_margin)
    st = cse.cse_platten_stats(P.handle)
    n, d = P.n_tiles, P.d
    dev = "cuda"
    o = P._alloc(dev)
    o.update(cp=torch.empty(n, dtype=torch.float64, device=dev),
             bound=torch.empty(n, dtype=torch.float64, device=dev))
    if calibrating:
        o.update(alpha_prime=torch.empty(n, dtype=torch.float64, device=dev),
                 k=torch.empty(n, dtype=torch.int32, device=dev),
                 lam=torch.empty(n, dtype=torch.float64, device=dev),
                 lam_g=torch.empty(1, dtype=torch.float64, device=dev),
                 rej_at=torch.empty(n, dtype=torch.int32, device=dev))

    if calibrating:
        def step():
            cse.cse_calibrate(P.handle, w["seed"], w["alpha"], o["alpha_prime"], o["k"], o["lam"], o["lam_g"],
                              o["rej_at"], w["delta"], o["reject"], o["score_T"], o["score_Z"], o["grad"],
                              o["cp"], o["bound"])
    else:
        def step():
            cse.cse_validate(P.handle, w["seed"], w["delta"], o["reject"], o["score_T"], o["score_Z"], o["grad"],
                             o["cp"], o["bound"])

    tune = None
    if args.autotune:
        t_tune = time.perf_counter()
        v, g = cse.cse_autotune(P.handle, seed=w["seed"])
        tune = {"value": v, "grid": g, "seconds": time.perf_counter() - t_tune}

    def note(msg):
        if args.progress:
            print(f"bench.py: {msg} ({time.perf_counter() - t_start:.1f} s)", file=sys.stderr, flush=True)

    t_start = time.perf_counter()
    note(f"platten of {P.n_tiles} tiles built in {platten_ms:.0f} ms")
    for i in range(warmup):
        step()
        if args.progress:
            torch.cuda.synchronize()
        note(f"warmup step {i + 1} done")
    torch.cuda.synchronize()
    cse.cse_profile_reset()
    cse.cse_profile_enable(True)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for i in range(steps):
        step()
        if args.progress:
            torch.cuda.synchronize()
        note(f"timed step {i + 1} done")
    torch.cuda.synchronize()
    dt = time.perf_counter() - t
    cse.cse_profile_enable(False)
    sim_kernel = {"binom2": "binom2", "hier4": "hier4", "ztest1": "ztest1", "phase23": "phase23",
                  "basket4": "basket4"}[design] + \
        ("_calib" if calibrating else "")
    kern = {}
    for kn in (sim_kernel, "select", "b2_bracket", "hier4_pilot", "h4_bracket", "bound_invert", "bound_validate"):
        cnt, ms = cse.cse_profile_get(kn)
        if cnt:
            kern[kn] = round(ms / cnt, 5)
    total = st["total_sims"] * steps
    value = total / dt
    ms_step = dt / steps * 1e3

    # the Taylor comparison bound and worst-case vertex (Section 4.3) from this step's outputs,
    # timed on its own (not part of the step)
    taylor = None
    if full and "grad" in o and o["grad"] is not None:
        cse.cse_profile_reset()
        cse.cse_profile_enable(True)
        for _ in range(5):
            to = P.taylor(o["cp"], o["grad"])
        torch.cuda.synchronize()
        cse.cse_profile_enable(False)
        cnt, ms = cse.cse_profile_get("taylor")
        taylor = {"kernel_ms": ms / max(cnt, 1), "max_bound": float(to["bound"].max().item()),
                  "max_tilt_bound": float(o["bound"].max().item())}

    # the two-sided band (Remark 2), a confidence set (Section 8) and the randomised calibration,
    # each on this step's outputs and timed on its own (not part of the step)
    ext = None
    if full and not args.no_extensions and n:
        ext = {}
        cse.cse_profile_reset()
        cse.cse_profile_enable(True)
        for _ in range(5):
            lo = P.validate_lower(o["reject"], delta=w["delta"])
        torch.cuda.synchronize()
        cnt, ms = cse.cse_profile_get("bound_lower")
        ext["lower_bound"] = {"kernel_ms": ms / max(cnt, 1), "min_lower": float(lo["lower"].min().item())}
        if calibrating:
            coef = [-1.0, 1.0] + [0.0] * (d - 2) + [0.0]      # e(theta) = theta_1 - theta_0
            for _ in range(5):
                cs = P.confidence_set(float(o["lam"].median().item()), o["lam"], coef)
            torch.cuda.synchronize()
            cnt, ms = cse.cse_profile_get("confidence_set")
            ext["confidence_set"] = {"ms": ms / max(cnt, 1), "kept": int(cs["keep"].sum().item()),
                                     "e_range": [float(x) for x in cs["e_range"].tolist()]}
            reps = steps if ms_step < 1000.0 else 1      # long steps: one call, no warm-up
            if reps > 1:
                tb = P.calibrate_tiebreak(w["seed"], alpha=w["alpha"])
                torch.cuda.synchronize()
            cse.cse_profile_reset()
            tt = time.perf_counter()
            for _ in range(reps):
                tb = P.calibrate_tiebreak(w["seed"], alpha=w["alpha"])
            torch.cuda.synchronize()
            dtt = (time.perf_counter() - tt) / reps
            cnt, ms = cse.cse_profile_get("tiebreak")
            ext["tiebreak"] = {"ms_per_step": dtt * 1e3, "kernel_ms": ms / max(cnt, 1),
                               "value": st["total_sims"] / dtt,
                               "same_lambda_as_plain": bool(torch.equal(tb["lambda_tile"], o["lam"])),
                               "step": "alpha' -> simulation -> selection -> tie-break, no validation bound"}
        cse.cse_profile_enable(False)

    # the same step captured once as a HIP graph and replayed (outputs checked against eager)
    graph = None
    if full and not args.no_graph:
        ref = {k: v.clone() for k, v in o.items() if v is not None}
        t_cap = time.perf_counter()
        if calibrating:
            plan = cse.cse_plan_calibrate(P.handle, w["seed"], w["alpha"], o["alpha_prime"], o["k"], o["lam"],
                                          o["lam_g"], o["rej_at"], w["delta"], o["reject"], o["score_T"],
                                          o["score_Z"], o["grad"], o["cp"], o["bound"])
        else:
            plan = cse.cse_plan_validate(P.handle, w["seed"], w["delta"], o["reject"], o["score_T"], o["score_Z"],
                                         o["grad"], o["cp"], o["bound"])
        cap_ms = (time.perf_counter() - t_cap) * 1e3
        cse.cse_plan_launch(plan)
        torch.cuda.synchronize()
        tg = time.perf_counter()
        for i in range(steps):
            cse.cse_plan_launch(plan)
            if args.progress:
                torch.cuda.synchronize()
            note(f"graph replay {i + 1} done")
        torch.cuda.synchronize()
        dtg = time.perf_counter() - tg
        same = all(torch.equal(ref[k], o[k]) for k in ref)
        graph = {"ms_per_step": dtg / steps * 1e3, "value": st["total_sims"] * steps / dtg,
                 "capture_ms": cap_ms, "nodes": cse.cse_plan_nodes(plan), "identical_to_eager": same}
        cse.cse_plan_destroy(plan)
        if not same:
            print("bench.py: graph replay outputs differ from the eager step", file=sys.stderr)
            sys.exit(1)

    # roofline of the dominant kernel: the fused simulation
    ops_min = None
    if design == "binom2":
        ops = (st["group_sims"] * (B2_PHILOX + B2_COUNT_G)
               + st["total_sims"] * (B2_TILE_CAL if calibrating else B2_TILE_FWD))
        ops_min = b2_method_min_ops(P, w, calibrating)
        kname = f"k_binom2<KEYS={'true' if calibrating else 'false'}>"
    elif design == "hier4":
        boxes = np.unique(P.tiles["box"])
        box_sims = int(np.asarray(w["sims"])[boxes].sum())
        ops = (st["group_sims"] * H4_PHILOX + st["batch_sims"] * H4_COUNT + box_sims * H4_BOX
               + st["total_sims"] * H4_TILE)
        kname = "k_hier4<1, false, true>"
        if args.h4_bracket:   # the timed kernel is the pass after the 2,048-simulation pilot
            sims = np.asarray(w["sims"])[boxes].astype(np.int64)
            ops = ops * float(np.maximum(sims - 2048, 0).sum()) / float(sims.sum())
            kname = "k_hier4<2, false, true>"
    elif design == "basket4":
        ops = st["group_sims"] * H4_PHILOX + st["batch_sims"] * H4_COUNT + st["total_sims"] * BK_SLOT
        kname = "k_hier4<0, true, true>"
    elif design == "phase23":
        wc = cse.cse_work_counters(P.handle)
        ops = (wc["looks_phase2"] * (90 * P23_NODE + P23_P2_EXTRA)
               + wc["looks_phase3"] * (90 * (P23_NODE + P23_TAIL) + P23_P3_EXTRA)
               + wc["newton_steps"] * P23_NEWTON)
        kname = "k_phase23"
    else:
        ops = None
        kname = "k_ztest1<KEYS=true>"
    k_s = kern.get(sim_kernel, 0.0) * 1e-3
    roof = None
    if ops is not None and k_s > 0:
        achieved = ops / k_s
        roof = {"bound": "alu", "achieved": achieved / 1e12, "peak": VALU_PEAK / 1e12,
                "unit": "Tops/s (float64 VALU)" if design == "phase23" else "Tops/s (int32 VALU)",
                "frac": achieved / VALU_PEAK, "traffic": None,
                "kernel": kname, "kernel_ms": kern[sim_kernel], "ops_per_launch": ops}
        if design == "phase23":
            roof["work"] = wc
        if ops_min is not None:
            roof["ops_method_minimal"] = ops_min
            roof["frac_method_minimal"] = ops_min / k_s / VALU_PEAK
        if name in TRAFFIC:
            roof["traffic"] = TRAFFIC[name]
            roof["traffic_unit"] = "bytes per launch"

    # the plain forward-only per-tile path, same tiles, seed and N: identical counts (equal bound)
    plain = None
    if not args.no_plain:
        R_plain = torch.empty(n, dtype=torch.int32, device=dev)
        cse.cse_simulate_per_tile(P.handle, w["seed"], 0, min(n, 64), R_plain)   # warm
        torch.cuda.synchronize()
        tp = time.perf_counter()
        cse.cse_simulate_per_tile(P.handle, w["seed"], 0, n, R_plain)
        torch.cuda.synchronize()
        dtp = time.perf_counter() - tp
        equal = bool(torch.equal(R_plain, o["reject"]))
        plain = {"value": st["total_sims"] / dtp, "unit": "sim·tiles/s", "ms": dtp * 1e3,
                 "path": "cse_simulate_per_tile: one launch per tile, forward counts only",
                 "identical_counts": equal}
        if not equal:
            print("bench.py: per-tile path counts differ from the fused path", file=sys.stderr)
            sys.exit(1)

    res = {
        "metric": METRIC, "value": value, "unit": "sim·tiles/s", "n_gpus": 1, "steps": steps,
        "warmup": warmup, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u32/f32/f64", "data": "synthetic",
        "config": {"workload": WORKLOADS[name], "name": name, "tiles": n,
                   "sims_per_tile": int(np.max(w["sims"])), "parallelism": "single GPU"},
        "speedup_vs_plain_fwd": (value / plain["value"]) if plain else None,
        "plain_fwd_per_tile": plain,
        "kernel_avg_ms": kern,
        "graph_replay": graph,
        "taylor": taylor,
        "extensions": ext,
        "autotune": tune,
        "launch_shape": cse.cse_platten_stats(P.handle)["launch_shape"],
        "platten_build_ms": platten_ms,
        "max_tile_bound": float(o["bound"].max().item()) if n else None,
        "roofline": roof,
    }
    if calibrating:
        res["lambda_global"] = float(o["lam_g"].item())
    if design in ("hier4", "phase23"):
        res["design_table_build_ms"] = st["table_build_us"] / 1e3
    P.close()
    return res


if __name__ == "__main__":
    main()
