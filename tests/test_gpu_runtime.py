"""GPU: platten creation and destruction as a runtime service.  Creation stages the read-only
per-tile arrays and design tables into one device transfer and takes its side stream from a
per-device cache that destroyed plattens refill; many plattens of different designs created
and destroyed in turn (and two alive at once) must give exactly the results of a platten
created alone, and every platten's calibration plan must replay identically."""
import numpy as np
import pytest
import torch

import paper_2212_10042_amd as cse
import workloads as W

pytestmark = pytest.mark.gpu


def _val(kind, w, seed=3):
    P = cse.Platten.create(kind, w["theta"], w["radii"], w["sims"])
    o = P.validate(seed, delta=0.01)
    torch.cuda.synchronize()
    out = {k: o[k].cpu().numpy().copy() for k in ("reject", "cp_upper", "tile_bound")}
    P.close()
    return out


def test_create_destroy_cycles_reproduce():
    b2 = W.binom2_grid(8, 512, lo=-2.0, hi=0.0, seed=1)
    h4 = W.hier4_grid(2, 64)
    zt = W.ztest_1d(16, 500, seed=2)
    ref = {"binom2": _val("binom2", b2), "hier4": _val("hier4", h4), "ztest1": _val("ztest1", zt)}
    print("[runtime] 30 create/validate/destroy cycles over three designs", flush=True)
    for i in range(30):
        kind, w = [("binom2", b2), ("hier4", h4), ("ztest1", zt)][i % 3]
        got = _val(kind, w)
        for k in ref[kind]:
            assert np.array_equal(got[k], ref[kind][k]), (i, kind, k)
    # two plattens alive at once (two side streams out of the cache), interleaved calls
    P = cse.Platten.create("binom2", b2["theta"], b2["radii"], b2["sims"])
    Q = cse.Platten.create("ztest1", zt["theta"], zt["radii"], zt["sims"])
    a = P.validate(3, delta=0.01)
    c = Q.validate(3, delta=0.01)
    torch.cuda.synchronize()
    assert np.array_equal(a["tile_bound"].cpu().numpy(), ref["binom2"]["tile_bound"])
    assert np.array_equal(c["tile_bound"].cpu().numpy(), ref["ztest1"]["tile_bound"])
    Q.close()
    P.close()


def test_plans_after_stream_reuse():
    """A calibration plan (the alpha' inversion and the validation bound are graph branches on
    the platten's side stream) captured on a platten whose side stream came from the cache."""
    w = W.binom2_grid(8, 512, lo=-2.0, hi=0.0, seed=1)
    for _ in range(3):   # put streams into the cache
        cse.Platten.create("binom2", w["theta"], w["radii"], w["sims"]).close()
    P = cse.Platten.create("binom2", w["theta"], w["radii"], w["sims"])
    e = P.calibrate(5, alpha=0.025, delta=0.01)
    torch.cuda.synchronize()
    ref = {k: v.clone() for k, v in e.items() if isinstance(v, torch.Tensor)}
    n = P.n_tiles
    o = {k: torch.empty_like(v) for k, v in ref.items()}
    plan = cse.cse_plan_calibrate(P.handle, 5, 0.025, o["alpha_prime"], o["k"], o["lambda_tile"],
                                  o["lambda_global"], o["reject_at_lambda"], 0.01, o.get("reject"),
                                  o.get("score_T"), o.get("score_Z"), o.get("grad"), o.get("cp_upper"),
                                  o.get("tile_bound"))
    for _ in range(3):
        for v in o.values():
            v.zero_()
        cse.cse_plan_launch(plan)
        torch.cuda.synchronize()
        for k in ref:
            assert torch.equal(o[k], ref[k]), k
    cse.cse_plan_destroy(plan)
    assert n > 0
    P.close()
