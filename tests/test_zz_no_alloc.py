"""GPU: cse_calibrate_noalloc (calibration keys in the library's static per-device workspace, no
allocation in the call) gives exactly cse_calibrate's outputs on the same platten, on two calls in a
row with the second platten smaller, and refuses a platten whose keys exceed the workspace."""
import numpy as np
import pytest
import torch

import workloads as W

pytestmark = pytest.mark.gpu

KEYS = ("reject", "score_T", "score_Z", "grad", "alpha_prime", "k", "lambda_tile", "lambda_global",
        "reject_at_lambda", "cp_upper", "tile_bound")


def _cases():
    import paper_2212_10042_amd as cse
    big = W.binom2_grid(20, 1000, seed=3)          # ragged 20 x 20 lower triangle, N = 1000
    small = W.binom2_grid(8, 300, seed=4)
    h4 = W.hier4_grid(3, 700)
    h4s = W.hier4_grid(2, 130)
    z = W.ztest_1d(64, 2000)
    zs = W.ztest_1d(16, 77)
    p23 = W.phase23_grid((2, 2, 2, 2), sims=300)
    p23s = W.phase23_grid((1, 2, 1, 2), sims=65)
    # the 4-arm calibration from bracketed keys (CSE_OPT_H4_BRACKET): small boxes (k > 0), N past
    # the 2,048-simulation pilot
    h4b = W.hier4_grid(2, 3000, lo=-0.08, hi=0.08, seed=6)
    h4bs = W.hier4_grid(2, 2500, lo=-0.06, hi=0.06, seed=7)
    return [("binom2", big, small), ("hier4", h4, h4s), ("ztest1", z, zs), ("phase23", p23, p23s),
            ("hier4+bracket", h4b, h4bs)], cse


def _run(P, noalloc, seed):
    o = P.calibrate(seed=seed, alpha=0.025, delta=0.01, noalloc=noalloc)
    torch.cuda.synchronize()
    return {k: (v.cpu().numpy() if v is not None else None) for k, v in o.items()}


@pytest.mark.parametrize("i", [0, 1, 2, 3, 4])
def test_noalloc_matches_calibrate_twice(i):
    torch.cuda.set_device(0)
    cases, cse = _cases()
    kind, first, second = cases[i]
    for w, seed in ((first, 11), (second, 12)):   # the second call on a smaller platten
        P = cse.Platten.create(kind.split("+")[0], w["theta"], w["radii"], w["sims"], cut=w.get("cut"))
        if kind.endswith("+bracket"):
            cse.cse_platten_set_option(P.handle, cse.CSE_OPT_H4_BRACKET, 1)
        print(f"noalloc case {kind}: {P.n_tiles} tiles, seed {seed}", flush=True)
        ref = _run(P, False, seed)
        got = _run(P, True, seed)
        for k in KEYS:
            if ref.get(k) is None:
                assert got.get(k) is None
                continue
            assert np.array_equal(ref[k], got[k]), f"{kind}: {k} differs between cse_calibrate and the no-alloc call"
        P.close()


def test_noalloc_refuses_oversized_platten():
    torch.cuda.set_device(0)
    import paper_2212_10042_amd as cse
    w = W.binom2_grid(256, 16384, seed=5)   # 32,896 tiles x 16,384 sims: records far above the workspace
    P = cse.Platten.create("binom2", w["theta"], w["radii"], w["sims"])
    assert cse.cse_platten_stats(P.handle)["n_key_slots"] * 16 > cse.NOALLOC_SCRATCH_BYTES
    with pytest.raises(cse.CseError) as e:
        P.calibrate(seed=1, noalloc=True)
    assert e.value.status == cse.CSE_EINVAL
    P.close()
