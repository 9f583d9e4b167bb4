"""GPU: calibration / validation steps captured as HIP graphs (cse_plan_*) and the launch-shape
autotuner (cse_autotune), for every design.

A plan must reproduce the eager call bit for bit on every replay, with the program's own eager
work (other calibrations on the same platten, fills, synchronisations) between replays.  The
autotuner may only change speed: outputs after tuning equal those before.
"""
import numpy as np
import pytest
import torch

import paper_2212_10042_amd as cse
import workloads as W

pytestmark = pytest.mark.gpu


def _case(kind):
    if kind == "ztest1":
        return W.ztest_1d(40, 3000)
    if kind == "binom2":
        return W.binom2_grid(24, 500)
    if kind == "hier4":
        return W.hier4_grid(2, 300)
    if kind == "basket4":
        return W.basket_grid(2, 300, lo=-2.4, hi=-0.9)
    w = W.phase23_grid((2, 2, 2, 1), 100)
    return w


KINDS = ["ztest1", "binom2", "hier4", "phase23", "basket4"]


def _alloc(P, dev="cuda"):
    n, d = P.n_tiles, P.d
    kind = P.design.kind
    o = dict(alpha_prime=torch.empty(n, dtype=torch.float64, device=dev),
             k=torch.empty(n, dtype=torch.int32, device=dev),
             lam=torch.empty(n, dtype=torch.float64, device=dev),
             lam_g=torch.empty(1, dtype=torch.float64, device=dev),
             rej_at=torch.empty(n, dtype=torch.int32, device=dev),
             reject=torch.empty(n, dtype=torch.int32, device=dev),
             cp=torch.empty(n, dtype=torch.float64, device=dev),
             bound=torch.empty(n, dtype=torch.float64, device=dev))
    o["score_T"] = (torch.empty((n, d), dtype=torch.int64, device=dev) if kind == cse.CSE_BINOM2_Z else
                    torch.empty((n, 2 * d), dtype=torch.int64, device=dev) if kind == cse.CSE_PHASE23 else None)
    o["score_Z"] = torch.empty(n, dtype=torch.float64, device=dev) if kind == cse.CSE_ZTEST1 else None
    o["grad"] = (torch.empty((n, d), dtype=torch.float64, device=dev)
                 if kind not in (cse.CSE_HIER4, cse.CSE_BASKET4) else None)
    return o


def _calib_args(o):
    return (o["alpha_prime"], o["k"], o["lam"], o["lam_g"], o["rej_at"], 0.01, o["reject"], o["score_T"],
            o["score_Z"], o["grad"], o["cp"], o["bound"])


def _eager(P, seed, o):
    cse.cse_calibrate(P.handle, seed, 0.025, *_calib_args(o))


def _fill(o):
    for t in o.values():
        if t is not None:
            t.fill_(-7)


def _same(a, b):
    for key in a:
        if a[key] is None:
            continue
        assert torch.equal(a[key], b[key]), key


def test_bracketed_hier4_plan_replays_match_eager():
    """The 4-arm calibration from bracketed keys captured as a graph (the inversion on a branch
    beside the pilot pass, the brackets after both): every replay equals the eager bracketed call
    and the every-key call, with eager work between replays."""
    w = W.hier4_grid(2, 3000, lo=-0.08, hi=0.08, seed=5)   # k > 0 on every tile, N > the pilot
    print("[graph] bracketed 4-arm calibration plan", flush=True)
    P = cse.Platten.create("hier4", w["theta"], w["radii"], w["sims"])
    every = _alloc(P)
    _eager(P, 3, every)
    cse.cse_platten_set_option(P.handle, cse.CSE_OPT_H4_BRACKET, 1)
    ref = _alloc(P)
    _eager(P, 3, ref)
    torch.cuda.synchronize()
    assert int(ref["k"].min().item()) > 0
    _same(every, ref)
    out = _alloc(P)
    other = _alloc(P)
    plan = cse.cse_plan_calibrate(P.handle, 3, 0.025, *_calib_args(out))
    try:
        for rep in range(3):
            _fill(out)
            cse.cse_plan_launch(plan)
            torch.cuda.synchronize()
            _same(ref, out)
            _eager(P, 100 + rep, other)
            torch.cuda.synchronize()
    finally:
        cse.cse_plan_destroy(plan)
    P.close()


@pytest.mark.parametrize("kind", KINDS)
def test_calibration_plan_replays_match_eager(kind):
    w = _case(kind)
    print(f"[graph] calibration plan {kind}", flush=True)
    P = cse.Platten.create(kind, w["theta"], w["radii"], w["sims"], cut=w.get("cut"))
    ref = _alloc(P)
    _eager(P, 3, ref)
    torch.cuda.synchronize()
    out = _alloc(P)
    other = _alloc(P)
    plan = cse.cse_plan_calibrate(P.handle, 3, 0.025, *_calib_args(out))
    try:
        assert cse.cse_plan_nodes(plan) > 0
        for rep in range(3):
            _fill(out)
            cse.cse_plan_launch(plan)
            torch.cuda.synchronize()
            _same(ref, out)
            # the program's own eager work between replays: another seed on the same platten
            _eager(P, 100 + rep, other)
            torch.cuda.synchronize()
    finally:
        cse.cse_plan_destroy(plan)
    P.close()


def test_validation_plan_replays_match_eager():
    w = W.binom2_grid(24, 700, lower_triangle=False)
    print("[graph] validation plan binom2 keep_all", flush=True)
    P = cse.Platten.create("binom2", w["theta"], w["radii"], w["sims"], keep_all=True)
    ref = P.validate(seed=5)
    torch.cuda.synchronize()
    o = P._alloc("cuda")
    o.update(cp_upper=torch.empty(P.n_tiles, dtype=torch.float64, device="cuda"),
             tile_bound=torch.empty(P.n_tiles, dtype=torch.float64, device="cuda"),
             q_star=torch.empty(P.n_tiles, dtype=torch.float64, device="cuda"))
    plan = cse.cse_plan_validate(P.handle, 5, 0.01, o["reject"], o["score_T"], o["score_Z"], o["grad"],
                                 o["cp_upper"], o["tile_bound"], o["q_star"])
    try:
        for rep in range(3):
            _fill(o)
            cse.cse_plan_launch(plan)
            torch.cuda.synchronize()
            _same(ref, o)
            P.validate(seed=50 + rep)
            torch.cuda.synchronize()
    finally:
        cse.cse_plan_destroy(plan)
    P.close()


@pytest.mark.parametrize("kind", KINDS)
def test_autotune_changes_speed_only(kind):
    w = _case(kind)
    print(f"[autotune] {kind}", flush=True)
    P = cse.Platten.create(kind, w["theta"], w["radii"], w["sims"], cut=w.get("cut"))
    ref = _alloc(P)
    _eager(P, 11, ref)
    torch.cuda.synchronize()
    value, grid = cse.cse_autotune(P.handle, seed=11, max_trials=20_000)
    st = cse.cse_platten_stats(P.handle)
    assert st["launch_shape"] == value
    print(f"[autotune] {kind}: chose {value} (grid {grid})", flush=True)
    out = _alloc(P)
    _eager(P, 11, out)
    torch.cuda.synchronize()
    _same(ref, out)
    P.close()


@pytest.mark.parametrize("kind", ["binom2", "phase23"])
def test_stale_plans_are_refused(kind):
    """A plan captured before cse_autotune rebuilt the launch shape, or one whose platten was
    destroyed, is refused by cse_plan_launch (CSE_EINVAL) and never replayed; a plan captured after
    tuning replays as usual."""
    w = _case(kind)
    print(f"[graph] stale plan {kind}", flush=True)
    P = cse.Platten.create(kind, w["theta"], w["radii"], w["sims"], cut=w.get("cut"))
    out = _alloc(P)
    plan = cse.cse_plan_calibrate(P.handle, 3, 0.025, *_calib_args(out))
    try:
        cse.cse_autotune(P.handle, seed=3, max_trials=5_000)
        torch.cuda.synchronize()
        with pytest.raises(cse.CseError) as e:
            cse.cse_plan_launch(plan)
        assert e.value.status == cse.CSE_EINVAL
    finally:
        cse.cse_plan_destroy(plan)
    fresh = cse.cse_plan_calibrate(P.handle, 3, 0.025, *_calib_args(out))
    cse.cse_plan_launch(fresh)
    torch.cuda.synchronize()
    ref = _alloc(P)
    _eager(P, 3, ref)
    torch.cuda.synchronize()
    _same(ref, out)
    P.close()
    with pytest.raises(cse.CseError) as e:
        cse.cse_plan_launch(fresh)
    assert e.value.status == cse.CSE_EINVAL
    cse.cse_plan_destroy(fresh)
