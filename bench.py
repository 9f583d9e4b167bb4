#!/usr/bin/env python3
"""Throughput of one step of the CSE hot path on one MI355X.

Workload: 2-arm binomial design (n = 35 per arm, pooled two-proportion z, reject z > 1.96),
256 x 256 boxes on logit [-3, 1]^2 kept to theta1 <= theta0 (32,896 tiles, 256 of them
triangles cut by the null boundary), 8,192 simulations per tile, seed 0.

One step = one call of cse_calibrate with every output requested: the inverted Tilt-Bound
target alpha'_i and k_i, the fused simulation (Philox common random numbers, draws, pooled z,
rejection counts at the fixed cut, score sums for the gradient, per-simulation calibration
keys), the order-statistic selection lambda*_i and its count below, lambda* = min, the
gradient, and the Clopper-Pearson + Tilt-Bound of every tile.  The platten (null clipping,
vertices, thresholds, batch plan) is built once before timing and reported separately.

Prints one JSON line.  --gpus above 1 is refused: this build runs on one GPU.
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
# Algorithmic integer work of the fused 2-arm kernel:
OPS_PHILOX_PER_SIM = 18 * 10 * 4       # per (workgroup, simulation): 18 blocks x 10 rounds x
                                       # (2 32x32->64 products + 2 xor3), shared by the 4 batches
OPS_COUNT_PER_SIM = 2 * 35 * 8 * 2     # per (batch, simulation): 70 words x 8 thresholds x (cmp+add)
OPS_PER_SIM_TILE = 5                   # decision, accumulate, key store


def cpu_baseline(w, target_s: float = 15.0):
    """The oracle as it stands (validation pass + calibration pass), on a sample of tiles."""
    import numpy as np

    import oracle as O
    import workloads as W

    rng = np.random.default_rng(1234)
    n = w["theta"].shape[0]

    def run(m):
        idx = np.sort(rng.choice(n, m, replace=False))
        s = W.subsample(w, idx)
        t = time.perf_counter()
        O.validate("binom2", s["theta"], s["radii"], s["sims"], w["seed"], w["delta"])
        O.calibrate("binom2", s["theta"], s["radii"], s["sims"], w["seed"], w["alpha"])
        return time.perf_counter() - t, int(s["sims"].sum())

    dt, st = run(8)
    m = int(min(n, max(8, 8 * target_s / max(dt, 1e-3))))
    dt, st = run(m)
    return {"value": st / dt, "unit": "sim·tiles/s", "cores": 1, "kind": "oracle",
            "sample": f"{m} tiles drawn uniformly (seed 1234) of the same workload, all 8,192 sims each; "
                      f"oracle validate + calibrate, {dt:.1f} s single-threaded"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--copy-probe", type=int, default=0,
                    help="only copy this many bytes device-to-device 3 times (scales HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build measures one GPU only (--gpus 1); multi-GPU sharding is described "
              "in DESIGN.md but not built", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2212_10042_amd as cse
    import workloads as W

    torch.cuda.set_device(0)
    if args.copy_probe:
        src = torch.ones(args.copy_probe // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": args.copy_probe, "copies": 3}), flush=True)
        return
    w = W.binom2_256_tri()
    t0 = time.perf_counter()
    P = cse.Platten.create("binom2", w["theta"], w["radii"], w["sims"])
    platten_ms = (time.perf_counter() - t0) * 1e3
    st = cse.cse_platten_stats(P.handle)
    n = P.n_tiles
    dev = "cuda"
    o = dict(alpha_prime=torch.empty(n, dtype=torch.float64, device=dev),
             k=torch.empty(n, dtype=torch.int32, device=dev),
             lam=torch.empty(n, dtype=torch.float64, device=dev),
             lam_g=torch.empty(1, dtype=torch.float64, device=dev),
             rej_at=torch.empty(n, dtype=torch.int32, device=dev),
             reject=torch.empty(n, dtype=torch.int32, device=dev),
             score_T=torch.empty((n, 2), dtype=torch.int64, device=dev),
             grad=torch.empty((n, 2), dtype=torch.float64, device=dev),
             cp=torch.empty(n, dtype=torch.float64, device=dev),
             bound=torch.empty(n, dtype=torch.float64, device=dev))

    def step():
        cse.cse_calibrate(P.handle, w["seed"], w["alpha"], o["alpha_prime"], o["k"], o["lam"], o["lam_g"],
                          o["rej_at"], w["delta"], o["reject"], o["score_T"], None, o["grad"], o["cp"],
                          o["bound"])

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    cse.cse_profile_reset()
    cse.cse_profile_enable(True)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t
    cse.cse_profile_enable(False)
    kern = {}
    for name in ("binom2_calib", "select", "bound_invert", "bound_validate", "cp_table"):
        cnt, ms = cse.cse_profile_get(name)
        kern[name] = round(ms / max(cnt, 1), 5)
    total = st["total_sims"] * args.steps
    value = total / dt
    ms_step = dt / args.steps * 1e3

    # roofline of the dominant kernel (fused simulation, calibration variant)
    ops = (st["group_sims"] * OPS_PHILOX_PER_SIM + st["batch_sims"] * OPS_COUNT_PER_SIM
           + st["total_sims"] * OPS_PER_SIM_TILE)
    k_s = kern["binom2_calib"] * 1e-3
    achieved = ops / k_s if k_s > 0 else 0.0
    roof = {"bound": "alu", "achieved": achieved / 1e12, "peak": VALU_PEAK / 1e12, "unit": "Tops/s (int32 VALU)",
            "frac": achieved / VALU_PEAK, "traffic": None, "kernel": "k_binom2<KEYS=true>",
            "kernel_ms": kern["binom2_calib"], "ops_per_launch": ops}

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

    cpu = None if args.no_cpu_baseline else cpu_baseline(w)
    res = {
        "metric": METRIC, "value": value, "unit": "sim·tiles/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u32/f64", "data": "synthetic",
        "config": {"workload": "binom2 n=35 pooled-z, 256x256 boxes on [-3,1]^2 kept to theta1<=theta0 "
                               "(32,896 tiles), 8,192 sims/tile, seed 0, alpha 0.025, delta 0.01",
                   "tiles": n, "sims_per_tile": 8192, "parallelism": "single GPU"},
        "speedup_vs_plain_fwd": (value / plain["value"]) if plain else None,
        "plain_fwd_per_tile": plain,
        "kernel_avg_ms": kern,
        "platten_build_ms": platten_ms,
        "lambda_global": float(o["lam_g"].item()),
        "max_tile_bound": float(o["bound"].max().item()),
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(res), flush=True)
    P.close()


if __name__ == "__main__":
    main()
