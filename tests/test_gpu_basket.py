"""GPU parity: the Bayesian basket design (Section 10.1's validation case study; four arms
against fixed rates p_0a, 85% posterior rule) through the C ABI vs the oracle.

Bars: the float32 posterior table equals the oracle's float64 statistic rounded to float32 on
> 99% of sampled outcomes (max |diff| < 2e-7); tiles (pieces of the boxes cut at the null
boundaries, their centres, half-widths and configurations) identical; R, k, lambda_i (float32
keys on both sides), #{S < lambda_i}, lambda* exact; bounds and alpha' within 1e-9.
"""
import numpy as np
import pytest
import torch

import oracle as O
import paper_2212_10042_amd as cse
import workloads as W

pytestmark = pytest.mark.gpu


def _np(t):
    return t.detach().cpu().numpy()


def test_posterior_table_vs_oracle():
    w = W.basket_grid(2, 64, lo=-2.5, hi=-1.0)
    t0 = np.array([-1.7, -1.2, -2.0, -1.5])
    P = cse.Platten.create("basket4", w["theta"], w["radii"], w["sims"], theta0=t0)
    tbl = _np(cse.cse_posterior_table(P.handle))
    torch.cuda.synchronize()
    rng = np.random.default_rng(0)
    idx = rng.integers(0, 36 ** 4, 2500)
    ref = O.basket_table(idx, 35, t0).astype(np.float32)
    got = tbl[idx]
    same = np.all(got == ref, axis=1)
    print(f"[basket] table: {same.mean():.4f} identical, max |diff| {np.abs(got - ref).max():.3g}", flush=True)
    assert same.mean() > 0.99 and np.abs(got - ref).max() < 2e-7
    P.close()
    # equal rates: exchangeable arms -> permuting the outcome permutes the statistics
    P = cse.Platten.create("basket4", w["theta"], w["radii"], w["sims"])
    tbl = _np(cse.cse_posterior_table(P.handle)).reshape(36, 36, 36, 36, 4)
    torch.cuda.synchronize()
    sw = np.transpose(tbl, (1, 0, 2, 3, 4))[..., [1, 0, 2, 3]]
    # equal up to the float64 summation order (a float32 rounding step at most)
    np.testing.assert_allclose(sw, tbl, rtol=2e-7, atol=1e-30)
    P.close()


def _compare(w, seed, theta0=None, cut=0.15):
    th, rd, sm = w["theta"], w["radii"], w["sims"]
    print(f"[basket] compare {w['name']} seed={seed}", flush=True)
    P = cse.Platten.create("basket4", th, rd, sm, cut=cut, theta0=theta0)
    pieces = O.basket_subboxes(th, rd, theta0)
    assert P.n_tiles == len(pieces)
    assert np.array_equal(P.tiles["box"], [q[0] for q in pieces])
    assert np.array_equal(P.tiles["cfg"], [q[1] for q in pieces])
    assert np.array_equal(P.tiles["theta"], np.array([q[2] for q in pieces]))
    assert np.array_equal(P.tiles["radii"], np.array([q[3] for q in pieces]))
    g = P.calibrate(seed, alpha=w["alpha"], delta=w["delta"])
    torch.cuda.synchronize()
    ov = O.validate("basket4", th, rd, sm, seed, w["delta"], cut=cut, theta0=theta0)
    oc = O.calibrate("basket4", th, rd, sm, seed, w["alpha"], cut=cut, key_dtype=np.float32, theta0=theta0)
    assert np.array_equal(_np(g["reject"]), ov["R"])
    # score sums (sum over rejecting simulations of the arm counts) and the score gradient
    assert np.array_equal(_np(g["score_T"]), ov["score"])
    cen = np.array([q[2] for q in pieces])
    go = O.score_gradient("basket4", cen, ov["R"], ov["score"], ov["N"])
    np.testing.assert_allclose(_np(g["grad"]), go, rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(_np(g["cp_upper"]), ov["cp"], rtol=1e-9)
    np.testing.assert_allclose(_np(g["tile_bound"]), ov["bound"], rtol=1e-9)
    np.testing.assert_allclose(_np(g["alpha_prime"]), oc["alpha_prime"], rtol=1e-9)
    k = _np(g["k"])
    frac = (oc["N"] + 1.0) * oc["alpha_prime"]
    near = np.abs(frac - np.round(frac)) < 1e-7
    assert np.all((k == oc["k"]) | near)
    same = k == oc["k"]
    assert np.array_equal(_np(g["lambda_tile"])[same], oc["lam"][same])
    assert np.array_equal(_np(g["reject_at_lambda"])[same], oc["reject_at_lam"][same])
    if same.all():
        assert float(_np(g["lambda_global"])[0]) == oc["lam_global"]
    print(f"[basket] {P.n_tiles} tiles, R total {int(ov['R'].sum())}", flush=True)
    P.close()
    return ov


def test_small_grid_straddling_boundaries():
    w = W.basket_grid(3, 400, lo=-2.6, hi=-0.8, seed=1)   # boxes straddle logit(0.15) = -1.7346
    ov = _compare(w, seed=1)
    assert ov["R"].sum() > 0 and len(ov["box"]) > len(w["theta"])


def test_unequal_rates_uneven_sims_other_cut():
    w = W.basket_grid(2, 1, lo=-2.4, hi=-0.9, seed=2)
    w["sims"] = np.array([1, 63, 64, 65, 255, 256, 257, 600, 1000, 40, 3, 128, 129, 511, 512, 700], np.int32)
    _compare(w, seed=2, theta0=[-1.5, -1.9, -1.2, -1.65], cut=0.25)


def test_per_tile_path_and_determinism():
    w = W.basket_grid(2, 300, lo=-2.4, hi=-0.9, seed=3)
    P = cse.Platten.create("basket4", w["theta"], w["radii"], w["sims"])
    print(f"[basket] per-tile path: {P.n_tiles} tiles", flush=True)
    a = P.simulate(seed=5)
    b = P.simulate(seed=5)
    R = torch.empty(P.n_tiles, dtype=torch.int32, device="cuda")
    cse.cse_simulate_per_tile(P.handle, 5, 0, P.n_tiles, R)
    torch.cuda.synchronize()
    assert torch.equal(a["reject"], b["reject"]) and torch.equal(R, a["reject"])
    assert int(R.sum()) > 0
    # the pass without score sums decides exactly as the pass with them
    R2 = torch.empty_like(R)
    cse.cse_simulate(P.handle, 5, R2)
    torch.cuda.synchronize()
    assert torch.equal(R2, R)
    with pytest.raises(cse.CseError):   # the z-test score is not a basket output
        cse.cse_simulate(P.handle, 5, R, None, torch.empty(P.n_tiles, dtype=torch.float64, device="cuda"))
    P.close()


def test_full_basket4_16_validation_sampled_boxes():
    """The bench's launch (16^4 boxes on [-3.5, 1]^4, 73,521 pieces x 32,768 simulations):
    every piece of sampled boxes (among them boxes cut at the boundaries) against the oracle;
    properties at every tile."""
    w = W.basket4_16()
    th, rd, sm = w["theta"], w["radii"], w["sims"]
    P = cse.Platten.create("basket4", th, rd, sm)
    print(f"[basket] full workload: {P.n_tiles} tiles", flush=True)
    assert P.n_tiles == 73521
    v = P.validate(w["seed"], delta=w["delta"])
    torch.cuda.synchronize()
    box = P.tiles["box"]
    rng = np.random.default_rng(2)
    counts = np.bincount(box, minlength=len(th))
    split = np.flatnonzero(counts > 1)
    pick = np.unique(np.concatenate([[box[0], box[-1]], rng.choice(split, 2, replace=False),
                                     rng.choice(np.unique(box), 2, replace=False)]))
    sub = W.subsample(w, pick)
    ov = O.validate("basket4", sub["theta"], sub["radii"], sub["sims"], w["seed"], w["delta"], cut=0.15)
    ids = np.concatenate([np.flatnonzero(box == b) for b in pick])
    print(f"[basket] {len(pick)} boxes, {len(ids)} pieces compared", flush=True)
    assert np.array_equal(_np(v["reject"])[ids], ov["R"])
    np.testing.assert_allclose(_np(v["cp_upper"])[ids], ov["cp"], rtol=1e-9)
    np.testing.assert_allclose(_np(v["tile_bound"])[ids], ov["bound"], rtol=1e-9)
    R = _np(v["reject"])
    assert np.all((R >= 0) & (R <= 32768))
    assert np.all(_np(v["tile_bound"]) >= _np(v["cp_upper"]) - 1e-15)
    P.close()
