"""GPU parity: Phase II/III selection design (Section 10.2 and its appendix) through the C ABI vs
the oracle.

Both sides evaluate every look's posterior in float64 (the GPU with structured Newton steps,
warm-started across nodes; the oracle with generic elimination), so trial paths agree unless a
decision statistic lies within rounding of a threshold; the statistic S is compared in float32
on both sides (the oracle's float64 value rounded first).  Rejection counts, the integer score
sums (observed counts and sample sizes over rejecting trials), k, lambda*_i and the counts
below it must agree exactly; the discordant-trial count is printed.
"""
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest
import torch

import oracle as O
import paper_2212_10042_amd as cse
import workloads as W

pytestmark = pytest.mark.gpu


def _np(t):
    return t.detach().cpu().numpy()


def _oracle_tiles(w, seed, lam):
    th, rd, sm = w["theta"], w["radii"], w["sims"]
    subs = O.subtiles("phase23", th, rd)
    box = np.array([s[0] for s in subs])
    cfg = np.array([s[1] for s in subs], np.int32)
    o = O.sim_phase23(th[box], cfg, sm[box], seed, lam, want_S=True, want_info=True)
    N = sm[box]
    S32 = o["S"].astype(np.float32)
    rej = [S32[t, : N[t]] < np.float32(lam) for t in range(len(subs))]
    R = np.array([r.sum() for r in rej])
    sY = np.array([o["info"][t, : N[t], 7:11][rej[t]].sum(0) for t in range(len(subs))]).reshape(-1, 4)
    sN = np.array([o["info"][t, : N[t], 3:7][rej[t]].sum(0) for t in range(len(subs))]).reshape(-1, 4)
    return subs, box, cfg, N, S32, R, sY, sN


def _compare(w, seed, lam):
    th, rd, sm = w["theta"], w["radii"], w["sims"]
    print(f"[phase23] compare {w['name']} seed={seed} lambda={lam}", flush=True)
    P = cse.Platten.create("phase23", th, rd, sm, cut=lam)
    subs, box, cfg, N, S32, R, sY, sN = _oracle_tiles(w, seed, lam)
    got = list(zip(P.tiles["box"].tolist(), P.tiles["cfg"].tolist()))
    assert got == [(int(s[0]), int(s[1])) for s in subs]
    g = P.calibrate(seed, alpha=w["alpha"], delta=w["delta"])
    torch.cuda.synchronize()
    Rg = _np(g["reject"])
    print(f"[phase23] {len(subs)} tiles, {int(N.sum())} trials, R total {int(R.sum())}, "
          f"tiles with discordant R {int(np.sum(Rg != R))}", flush=True)
    assert np.array_equal(Rg, R)
    sc = _np(g["score_T"])
    assert np.array_equal(sc[:, :4], sY) and np.array_equal(sc[:, 4:], sN)
    p = 1.0 / (1.0 + np.exp(-th[box]))
    np.testing.assert_allclose(_np(g["grad"]), (sY - sN * p) / N[:, None], rtol=1e-12, atol=1e-15)
    cp = O.cp_upper(R, N, w["delta"])
    V = O._pad_vertices(subs, th)
    ub, _ = O.tile_bound("binom", th[box], V, cp, n=350)
    np.testing.assert_allclose(_np(g["cp_upper"]), cp, rtol=1e-9)
    np.testing.assert_allclose(_np(g["tile_bound"]), ub, rtol=1e-9)
    ap, _ = O.tile_inverse("binom", th[box], V, w["alpha"], n=350)
    np.testing.assert_allclose(_np(g["alpha_prime"]), ap, rtol=1e-9)
    k = np.floor((N + 1.0) * ap).astype(np.int64)
    frac = (N + 1.0) * ap
    near = np.abs(frac - np.round(frac)) < 1e-7
    kg = _np(g["k"])
    assert np.all((kg == k) | near)
    same = kg == k
    lam_o = np.array([O.order_statistic(S32[t, : N[t]], int(k[t])) for t in range(len(subs))])
    rej_o = np.array([int(np.sum(S32[t, : N[t]] < np.float32(lam_o[t]))) for t in range(len(subs))])
    lg = _np(g["lambda_tile"])
    assert np.array_equal(lg[same], lam_o[same])
    assert np.array_equal(_np(g["reject_at_lambda"])[same], rej_o[same])
    assert float(_np(g["lambda_global"])[0]) == lg.min()
    P.close()
    return len(subs), R


def test_phase23_small_grid_parity():
    w = W.phase23_grid((3, 3, 3, 3), 48, seed=1)
    n, R = _compare(w, seed=1, lam=w["cut"])
    assert n > 81 and R.sum() > 0


def test_phase23_uneven_sims_item_boundaries():
    """Tiles of 1, 63, 64, 65, 255, 256, 257 and 600 trials: the queue's 256-trial items, their
    tails, and lanes refilled across items and tiles."""
    w = W.phase23_grid((2, 2, 2, 1), 1, lo=-0.3, hi=0.6, seed=7)
    w["sims"] = np.array([1, 63, 64, 65, 255, 256, 257, 600], np.int32)
    _compare(w, seed=7, lam=0.1)


def test_phase23_per_tile_path_and_determinism():
    w = W.phase23_grid((2, 2, 2, 2), 200, seed=3)
    P = cse.Platten.create("phase23", w["theta"], w["radii"], w["sims"], cut=0.2)
    print(f"[phase23] per-tile path: {P.n_tiles} tiles", flush=True)
    a = P.simulate(seed=5)
    b = P.simulate(seed=5)
    R = torch.empty(P.n_tiles, dtype=torch.int32, device="cuda")
    cse.cse_simulate_per_tile(P.handle, 5, 0, P.n_tiles, R)
    torch.cuda.synchronize()
    assert torch.equal(a["reject"], b["reject"]) and torch.equal(a["score_T"], b["score_T"])
    assert torch.equal(R, a["reject"])
    assert int(R.sum()) > 0
    P.close()


def test_phase23_large_tiles_selection_paths():
    """Tiles above the 2,048-trial sample of the float32 selection: the bracket path, and tiles
    whose k-th smallest key is +inf among thousands of +inf keys (the candidate list overflows
    and the exact radix passes over all keys run)."""
    w = W.phase23_grid((2, 1, 1, 1), 1, lo=-0.2, hi=0.2, seed=9)
    w["theta"] = np.array([[0.6, -0.5, -0.5, -0.5], [0.1, 0.1, 0.1, 0.1]])
    w["radii"] = np.full((2, 4), 0.05)
    w["sims"] = np.array([5000, 2200], np.int32)
    n, R = _compare(w, seed=9, lam=0.06253)


def test_phase23_exchangeable_arms_tie_exactly():
    """Treatment arms with equal true rates: their data tie often, and then their posterior
    summaries must be bit-identical so that the selection keeps the first of the tied arms on
    both sides (the kernel's batched reciprocals preserve that symmetry)."""
    w = W.phase23_grid((1, 1, 1, 1), 1, seed=2)
    w["theta"] = np.array([[0.4, 0.0, 0.0, 0.0], [0.1, -0.3, -0.3, -0.3], [0.6, 0.3, 0.3, -0.2]])
    w["radii"] = np.full((3, 4), 0.05)
    w["sims"] = np.array([1500, 1500, 1500], np.int32)
    w["name"] = "phase23_exchangeable_arms"
    n, R = _compare(w, seed=2, lam=0.1)
    assert n == 3 and R.sum() > 0


def test_phase23_full_c5_sampled_boxes():
    """The bench's full Phase II/III launch (2^18 boxes, 2,048 .. 65,536 trials each, one
    calibration step with validation and gradient): every tile of one sampled box from each of
    the six trial-count classes against the oracle (~0.6 ms per trial, boxes in parallel
    threads); properties at every tile."""
    w = W.phase23_c5()
    th, rd, sm = w["theta"], w["radii"], w["sims"]
    P = cse.Platten.create("phase23", th, rd, sm, cut=w["cut"])
    print(f"[phase23] full C5: {P.n_tiles} tiles, {int(sm[P.tiles['box']].sum())} trials", flush=True)
    g = P.calibrate(w["seed"], alpha=w["alpha"], delta=w["delta"])
    torch.cuda.synchronize()
    print("[phase23] full C5 step done", flush=True)
    box = P.tiles["box"]
    rng = np.random.default_rng(5)
    counts = np.bincount(box, minlength=th.shape[0])
    pick = []
    for cls in sorted(set(sm.tolist())):   # one single-tile box per class of N
        cand = np.flatnonzero((sm == cls) & (counts == 1))
        pick.append(int(rng.choice(cand)))
    pick = np.array(sorted(pick))
    O.sim_phase23(th[pick[:1]], np.array([7], np.int32), np.array([1], np.int32), 1, w["cut"])  # rule constants

    def one(b):
        return _oracle_tiles(W.subsample(w, [b]), w["seed"], w["cut"])

    with ThreadPoolExecutor(len(pick)) as ex:
        res = list(ex.map(one, pick))
    for b, (subs, obox, cfg, N, S32, R, sY, sN) in zip(pick, res):
        ids = np.flatnonzero(box == b)
        assert len(ids) == len(subs) == 1
        assert np.array_equal(P.tiles["cfg"][ids], cfg)
        Rg = _np(g["reject"])[ids]
        print(f"[phase23] box {b}: N {int(N[0])}, R {int(R[0])} (GPU {int(Rg[0])})", flush=True)
        assert np.array_equal(Rg, R)
        sc = _np(g["score_T"])[ids]
        assert np.array_equal(sc[:, :4], sY) and np.array_equal(sc[:, 4:], sN)
        oc_ap, _ = O.tile_inverse("binom", th[[b]], O._pad_vertices(subs, th[[b]]), w["alpha"], n=350)
        np.testing.assert_allclose(_np(g["alpha_prime"])[ids], oc_ap, rtol=1e-9)
        frac = (N + 1.0) * oc_ap
        k = np.floor(frac).astype(np.int64)
        kg = _np(g["k"])[ids]
        assert np.all((kg == k) | (np.abs(frac - np.round(frac)) < 1e-7))
        if kg[0] == k[0]:
            lam_o = O.order_statistic(S32[0, : N[0]], int(k[0]))
            assert _np(g["lambda_tile"])[ids][0] == lam_o
            below = int(np.sum(S32[0, : N[0]] < np.float32(lam_o)))
            assert _np(g["reject_at_lambda"])[ids][0] == below
    # every tile: counts within N, the global threshold is the minimum
    Rall = _np(g["reject"])
    assert np.all((Rall >= 0) & (Rall <= sm[box]))
    lam = _np(g["lambda_tile"])
    assert float(_np(g["lambda_global"])[0]) == lam.min()
    P.close()
