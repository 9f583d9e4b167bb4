"""GPU parity: 2-arm binomial design (pooled z, n = 35) through the C ABI vs the CPU oracle.

Bar: integers (rejections, score sums, k, counts below lambda*) bit-exact; lambda*_i exact
(the statistic table is float64 on both sides); float64 bounds within 1e-9 relative
(different optimiser round-off on the same golden-section search).
"""
import math

import numpy as np
import pytest
import torch

import oracle as O
import paper_2212_10042_amd as cse
import workloads as W

pytestmark = pytest.mark.gpu

RTOL_BOUND = 1e-9


def _np(t):
    return t.detach().cpu().numpy()


def _tiles_match(P, subs):
    got = list(zip(P.tiles["box"].tolist(), P.tiles["cfg"].tolist()))
    want = [(int(s[0]), int(s[1])) for s in subs]
    assert got == want
    assert np.array_equal(P.tiles["n_vert"], [len(s[2]) for s in subs])


def _check_k(k_gpu, k_orc, ap_orc, N):
    frac = (N + 1.0) * ap_orc
    near = np.abs(frac - np.round(frac)) < 1e-7
    assert np.all((k_gpu == k_orc) | near)


def _full_compare(w, seed, keep_all=False):
    th, rd, sm = w["theta"], w["radii"], w["sims"]
    print(f"[binom2] compare {w['name']} seed={seed} tiles={th.shape[0]}", flush=True)
    P = cse.Platten.create("binom2", th, rd, sm, keep_all=keep_all)
    ov = O.validate("binom2", th, rd, sm, seed, w["delta"], keep_all=keep_all)
    oc = O.calibrate("binom2", th, rd, sm, seed, w["alpha"], keep_all=keep_all)
    _tiles_match(P, ov["subs"])
    g = P.calibrate(seed, alpha=w["alpha"], delta=w["delta"])
    torch.cuda.synchronize()
    box = ov["box"]
    assert np.array_equal(_np(g["reject"]), ov["R"])
    assert np.array_equal(_np(g["score_T"]), ov["score_box"][box])
    gr = O.score_gradient("binom2", th[box], ov["R"], ov["score_box"][box], ov["N"])
    np.testing.assert_allclose(_np(g["grad"]), gr, rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(_np(g["cp_upper"]), ov["cp"], rtol=RTOL_BOUND)
    np.testing.assert_allclose(_np(g["tile_bound"]), ov["bound"], rtol=RTOL_BOUND)
    np.testing.assert_allclose(_np(g["alpha_prime"]), oc["alpha_prime"], rtol=RTOL_BOUND)
    _check_k(_np(g["k"]), oc["k"], oc["alpha_prime"], oc["N"])
    same_k = _np(g["k"]) == oc["k"]
    assert np.array_equal(_np(g["lambda_tile"])[same_k], oc["lam"][same_k])
    assert np.array_equal(_np(g["reject_at_lambda"])[same_k], oc["reject_at_lam"][same_k])
    assert float(_np(g["lambda_global"])[0]) == oc["lam_global"]
    # validate entry point agrees with the calibrate pass
    v = P.validate(seed, delta=w["delta"])
    torch.cuda.synchronize()
    assert np.array_equal(_np(v["reject"]), ov["R"])
    np.testing.assert_allclose(_np(v["tile_bound"]), ov["bound"], rtol=RTOL_BOUND)
    P.close()


def test_small_lower_triangle_ragged():
    # 20 x 20 boxes: 8x8 tile batches with ragged edges; 1000 sims: ragged last wave chunk
    _full_compare(W.binom2_grid(20, 1000, seed=3), seed=3)


def test_keep_all_square_uneven_sims():
    w = W.binom2_grid(12, 300, lower_triangle=False, seed=5)
    w["sims"] = W.uneven_sims(w["theta"].shape[0], seed=1, lo_pow=5, n_classes=4)  # 32..256
    _full_compare(w, seed=5, keep_all=True)


def test_repeated_grid_points_and_partial_squares():
    """Boxes that share a grid point (the same centre three times, another twice) and a grid
    whose 4 x 4 squares of 8 x 8 batches are only partly filled (17 x 13 boxes, some with a
    different N): the workgroup items open extra squares for the repeated points and leave
    empty batches idle, with exact results."""
    w = W.binom2_grid(17, 700, lower_triangle=False, seed=11)
    th, rd, sm = w["theta"], w["radii"], w["sims"]
    rep = np.array([5, 5, 5, 100, 100])
    w["theta"] = np.concatenate([th, th[rep]])
    w["radii"] = np.concatenate([rd, rd[rep]])
    sims = np.concatenate([sm, sm[rep]])
    sims[::7] = 400   # a second N class
    w["sims"] = sims.astype(np.int32)
    _full_compare(w, seed=11, keep_all=True)


def test_edge_single_tile_and_one_sim():
    for sims in (1, 63, 64, 65):
        w = dict(name=f"single{sims}", theta=np.array([[0.25, -0.5]]), radii=np.array([[0.125, 0.125]]),
                 sims=np.array([sims], np.int32), delta=0.01, alpha=0.3)
        _full_compare(w, seed=11)


def test_edge_extreme_logits():
    # thresholds clamp at 0 and 2^32-1 in the corners of a wide grid
    w = W.binom2_grid(16, 200, lo=-40.0, hi=40.0, seed=2)
    _full_compare(w, seed=2)


def test_full_size_workload_sampled_tiles():
    """256x256 lower-triangle grid, 8,192 sims (the benchmark's launch), oracle on sampled tiles."""
    w = W.binom2_256_tri()
    th, rd, sm = w["theta"], w["radii"], w["sims"]
    P = cse.Platten.create("binom2", th, rd, sm)
    g = P.calibrate(w["seed"], alpha=w["alpha"], delta=w["delta"])
    torch.cuda.synchronize()
    n = th.shape[0]
    rng = np.random.default_rng(0)
    diag = np.flatnonzero(th[:, 0] == th[:, 1])
    idx = np.unique(np.concatenate([[0, n - 1], diag[[0, 100, 255]], rng.choice(n, 40, replace=False)]))
    print(f"[binom2] full-size sampled tiles: {idx.size}", flush=True)
    sub = W.subsample(w, idx)
    oc = O.calibrate("binom2", sub["theta"], sub["radii"], sub["sims"], w["seed"], w["alpha"])
    ov = O.validate("binom2", sub["theta"], sub["radii"], sub["sims"], w["seed"], w["delta"])
    # every box of this workload has exactly one tile, in box order
    assert P.n_tiles == n and np.array_equal(P.tiles["box"], np.arange(n))
    assert np.array_equal(_np(g["reject"])[idx], ov["R"])
    assert np.array_equal(_np(g["score_T"])[idx], ov["score_box"])
    np.testing.assert_allclose(_np(g["tile_bound"])[idx], ov["bound"], rtol=RTOL_BOUND)
    np.testing.assert_allclose(_np(g["alpha_prime"])[idx], oc["alpha_prime"], rtol=RTOL_BOUND)
    _check_k(_np(g["k"])[idx], oc["k"], oc["alpha_prime"], oc["N"])
    same = _np(g["k"])[idx] == oc["k"]
    assert np.array_equal(_np(g["lambda_tile"])[idx][same], oc["lam"][same])
    assert np.array_equal(_np(g["reject_at_lambda"])[idx][same], oc["reject_at_lam"][same])
    # properties at every tile: lambda* is the global min; counts below it are < k <= N
    lam = _np(g["lambda_tile"])
    assert float(_np(g["lambda_global"])[0]) == lam.min()
    assert np.all(_np(g["reject_at_lambda"]) < _np(g["k"]))
    assert np.all((_np(g["tile_bound"]) >= _np(g["cp_upper"])) & (_np(g["tile_bound"]) <= 1.0))
    P.close()


def test_per_tile_path_and_determinism():
    w = W.binom2_grid(24, 700, seed=9)
    P = cse.Platten.create("binom2", w["theta"], w["radii"], w["sims"])
    a = P.simulate(9)
    b = P.simulate(9)
    plain = torch.empty(P.n_tiles, dtype=torch.int32, device="cuda")
    cse.cse_simulate_per_tile(P.handle, 9, 0, P.n_tiles, plain)
    torch.cuda.synchronize()
    assert torch.equal(a["reject"], b["reject"]) and torch.equal(a["score_T"], b["score_T"])
    assert torch.equal(a["reject"], plain)
    c1 = P.calibrate(9)
    c2 = P.calibrate(9)
    torch.cuda.synchronize()
    for key in ("lambda_tile", "reject_at_lambda", "k", "reject", "score_T"):
        assert torch.equal(c1[key], c2[key])
    P.close()


def test_tie_autograd_matches_score_and_exact_gradient():
    w = W.binom2_grid(8, 20000, lo=-1.0, hi=1.0, lower_triangle=False, seed=0)
    th = torch.tensor(w["theta"], dtype=torch.float64, device="cuda", requires_grad=True)
    f = cse.TIE.apply(th, w["radii"], w["sims"], "binom2", 0)
    f.sum().backward()
    R, sT, _ = O.sim_binom2(w["theta"], w["sims"], 0)
    assert np.array_equal(np.round(_np(f) * w["sims"]).astype(np.int64), R)
    g_orc = O.score_gradient("binom2", w["theta"], R, sT, w["sims"])
    np.testing.assert_allclose(_np(th.grad), g_orc, rtol=1e-12, atol=1e-15)


def test_score_gradient_vs_central_differences_crn():
    """Central differences under common random numbers (h = 1e-3) against the score
    estimate; tolerance from the per-simulation spread of the score terms."""
    N = 16384
    pts = np.array([[0.0, 0.0], [-0.5, -0.75], [0.25, -1.0]])
    h = 1e-3
    rows = [pts]
    for a in range(2):
        for sgn in (1, -1):
            q = pts.copy()
            q[:, a] += sgn * h
            rows.append(q)
    allp = np.concatenate(rows)
    sims = np.full(allp.shape[0], N, np.int32)
    th = torch.tensor(allp, dtype=torch.float64, device="cuda", requires_grad=True)
    f = cse.TIE.apply(th, np.full_like(allp, 1e-3), sims, "binom2", 7)
    f.sum().backward()
    f = _np(f)
    g = _np(th.grad)[: pts.shape[0]]
    m = pts.shape[0]
    for a in range(2):
        fd = (f[m * (1 + 2 * a): m * (2 + 2 * a)] - f[m * (2 + 2 * a): m * (3 + 2 * a)]) / (2 * h)
        # score terms are bounded by 35 in magnitude; FD noise under CRN is ~ sqrt(#flips)/(N 2h)
        flips = np.abs(fd) * N * 2 * h + 1.0
        tol = 5 * (35 / math.sqrt(N)) + 5 * np.sqrt(flips) / (N * 2 * h)
        assert np.all(np.abs(fd - g[:, a]) <= tol)


def test_cse_bound_modes_vs_oracle():
    """cse_bound without simulation: mode 0 (CP + tilt) for arbitrary counts including R = 0 and
    R = N, mode 1 (alpha'), mode 2 (tilt of a given f(theta_i))."""
    w = W.binom2_grid(12, 999, seed=0)
    th, rd, sm = w["theta"], w["radii"], w["sims"]
    P = cse.Platten.create("binom2", th, rd, sm)
    n = P.n_tiles
    rng = np.random.default_rng(5)
    R = rng.integers(0, 999, n).astype(np.int32)
    R[:3] = [0, 999, 998]
    Rt = torch.tensor(R, device="cuda")
    a = rng.uniform(0.0, 0.3, n)
    a[:2] = [0.0, 1.0]
    at = torch.tensor(a, device="cuda")
    b0, _ = P.bound(0, R=Rt, level=0.05)
    b1, _ = P.bound(1, level=0.1)
    b2, _ = P.bound(2, a=at)
    torch.cuda.synchronize()
    subs = O.subtiles("binom2", th, rd)
    V = O._pad_vertices(subs, th)
    box = np.array([s[0] for s in subs])
    cp = O.cp_upper(R, sm[box], 0.05)
    e0, _ = O.tile_bound("binom", th[box], V, cp)
    e1, _ = O.tile_inverse("binom", th[box], V, 0.1)
    e2, _ = O.tile_bound("binom", th[box], V, a)
    np.testing.assert_allclose(_np(b0), e0, rtol=RTOL_BOUND)
    np.testing.assert_allclose(_np(b1), e1, rtol=RTOL_BOUND)
    np.testing.assert_allclose(_np(b2), e2, rtol=RTOL_BOUND, atol=1e-300)
    assert _np(b0)[1] == 1.0 and _np(b2)[0] == 0.0 and _np(b2)[1] == 1.0
    P.close()


def test_paper_worked_value_through_gpu_bound():
    """The optimized Tilt-Bound of the z-test at theta0 = -0.25, v = 0.25 with the exact
    f(theta0) is 2.73% (Section 4.3); the GPU bound kernel on the tile [-0.5, 0] reproduces it."""
    from scipy import stats
    P = cse.Platten.create("ztest1", np.array([[-0.25]]), np.array([[0.25]]), np.array([100], np.int32))
    f0 = stats.norm.cdf(-0.25 - stats.norm.ppf(0.975))
    b, _ = P.bound(2, a=torch.tensor([f0], device="cuda"))
    torch.cuda.synchronize()
    assert round(100 * float(_np(b)[0]), 2) == 2.73
    L = -math.log(f0)
    assert float(_np(b)[0]) == pytest.approx(math.exp(-(math.sqrt(L) - 0.25 / math.sqrt(2)) ** 2), rel=1e-10)
    P.close()


def test_full_c3_forward_gradient_sampled_and_fd():
    """All 1024^2 boxes on [-3,1]^2 with 16,384 sims (the 2^20-tile forward + gradient launch):
    R, score sums, gradient and bound vs the oracle on sampled tiles; the score gradient vs
    central differences under common random numbers (h = 1e-3) on every 256th tile."""
    w = W.binom2_1024_full()
    th, rd, sm = w["theta"], w["radii"], w["sims"]
    P = cse.Platten.create("binom2", th, rd, sm, keep_all=True)
    n = P.n_tiles
    assert n == 1 << 20
    g = P.validate(w["seed"], delta=w["delta"])
    torch.cuda.synchronize()
    rng = np.random.default_rng(3)
    idx = np.unique(np.concatenate([[0, n - 1, n // 2], rng.choice(n, 24, replace=False)]))
    print(f"[binom2] 2^20-tile launch, {idx.size} sampled tiles", flush=True)
    sub = W.subsample(w, idx)
    ov = O.validate("binom2", sub["theta"], sub["radii"], sub["sims"], w["seed"], w["delta"], keep_all=True)
    assert np.array_equal(_np(g["reject"])[idx], ov["R"])
    assert np.array_equal(_np(g["score_T"])[idx], ov["score_box"])
    go = O.score_gradient("binom2", sub["theta"], ov["R"], ov["score_box"], sub["sims"])
    np.testing.assert_allclose(_np(g["grad"])[idx], go, rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(_np(g["tile_bound"])[idx], ov["bound"], rtol=RTOL_BOUND)
    P.close()
    # central differences on every 256th tile, same seed (common random numbers)
    sel = np.arange(0, n, 256)
    h = 1e-3
    pts = th[sel]
    rows = [pts]
    for a in range(2):
        for sgn in (1, -1):
            q = pts.copy()
            q[:, a] += sgn * h
            rows.append(q)
    allp = np.concatenate(rows)
    N = int(sm[0])
    Q = cse.Platten.create("binom2", allp, np.full_like(allp, rd[0, 0]), np.full(allp.shape[0], N, np.int32),
                           keep_all=True)
    o = Q.simulate(w["seed"])
    torch.cuda.synchronize()
    f = _np(o["reject"]).astype(np.float64) / N
    m = sel.size
    gs = _np(g["grad"])[sel]
    for a in range(2):
        fd = (f[m * (1 + 2 * a): m * (2 + 2 * a)] - f[m * (2 + 2 * a): m * (3 + 2 * a)]) / (2 * h)
        flips = np.abs(fd) * N * 2 * h + 1.0
        tol = 5 * (35 / math.sqrt(N)) + 5 * np.sqrt(flips) / (N * 2 * h)
        d = fd - gs[:, a]
        assert np.all(np.abs(d) <= tol)
        z = d.mean() / (d.std(ddof=1) / math.sqrt(m))
        print(f"[binom2] FD vs score, arm {a}: mean diff {d.mean():.2e}, z {z:.2f} over {m} tiles", flush=True)
        assert abs(z) < 5
    Q.close()


def test_bound_search_paths_agree():
    """The float64 search over q takes eight lanes per tile (a parallel section search) on
    plattens below 2^18 tiles and one lane per tile (Brent's search) from 2^18 tiles on.  Each
    returns the best point it evaluated; on the same tiles alpha' (inversion) and the
    validation bound agree within 1e-9 relative."""
    w = W.binom2_grid(512, 1000, lower_triangle=False)
    P = cse.Platten.create("binom2", w["theta"], w["radii"], w["sims"], keep_all=True)
    assert P.n_tiles >= 1 << 18
    idx = np.arange(0, w["theta"].shape[0], 97)
    s = W.subsample(w, idx)
    Q = cse.Platten.create("binom2", s["theta"], s["radii"], s["sims"], keep_all=True)
    assert Q.n_tiles < 1 << 18
    print(f"[binom2] bound search paths: {P.n_tiles} vs {Q.n_tiles} tiles", flush=True)
    bp, bq = P.tiles["box"], Q.tiles["box"]
    assert np.array_equal(bp, np.arange(P.n_tiles)) and np.array_equal(bq, np.arange(Q.n_tiles))
    ap, _ = P.bound(1, level=0.025)
    aq, _ = Q.bound(1, level=0.025)
    Rp = torch.tensor((np.arange(P.n_tiles) * 7) % 100, dtype=torch.int32, device="cuda")
    Rq = torch.tensor((idx * 7) % 100, dtype=torch.int32, device="cuda")
    up, _ = P.bound(0, R=Rp, level=0.01)
    uq, _ = Q.bound(0, R=Rq, level=0.01)
    torch.cuda.synchronize()
    np.testing.assert_allclose(_np(ap)[idx], _np(aq), rtol=1e-9)
    np.testing.assert_allclose(_np(up)[idx], _np(uq), rtol=1e-9)
    P.close()
    Q.close()


@pytest.mark.parametrize("margin", [0.0, 100.0])
def test_selection_exact_pass_forced(margin):
    """The bracketed selection with a zero margin (most tiles' k-th statistic falls outside the
    bracket) or a very wide one (the batches' brackets overflow the LDS histogram): those tiles
    take the exact full-histogram pass, and lambda*_i and the counts below it still equal the
    oracle's and the default margin's; cse_work_counters counts the tiles sent there."""
    w = W.binom2_grid(16, 3000, lo=-2.0, hi=0.5, seed=7)
    th, rd, sm = w["theta"], w["radii"], w["sims"]
    print(f"[binom2] exact selection pass, margin {margin}", flush=True)
    P = cse.Platten.create("binom2", th, rd, sm)
    g0 = P.calibrate(7, alpha=0.05, with_validation=False)
    torch.cuda.synchronize()
    n0 = cse.cse_work_counters(P.handle)["trials"]
    cse.cse_platten_set_option(P.handle, cse.CSE_OPT_B2_MARGIN, margin)
    g1 = P.calibrate(7, alpha=0.05, with_validation=False)
    torch.cuda.synchronize()
    n1 = cse.cse_work_counters(P.handle)["trials"]
    print(f"[binom2] tiles in the exact pass: {n0} at the default margin, {n1} at {margin}", flush=True)
    assert n1 > n0
    if margin == 0.0:
        assert n1 >= P.n_tiles // 4
    for key in ("lambda_tile", "reject_at_lambda", "k"):
        assert np.array_equal(_np(g1[key]), _np(g0[key]))
    assert float(_np(g1["lambda_global"])[0]) == float(_np(g0["lambda_global"])[0])
    oc = O.calibrate("binom2", th, rd, sm, 7, 0.05)
    _check_k(_np(g1["k"]), oc["k"], oc["alpha_prime"], oc["N"])
    same_k = _np(g1["k"]) == oc["k"]
    assert np.array_equal(_np(g1["lambda_tile"])[same_k], oc["lam"][same_k])
    assert np.array_equal(_np(g1["reject_at_lambda"])[same_k], oc["reject_at_lam"][same_k])
    with pytest.raises(cse.CseError):
        cse.cse_platten_set_option(P.handle, cse.CSE_OPT_B2_MARGIN, -1.0)
    with pytest.raises(cse.CseError):
        cse.cse_platten_set_option(P.handle, 99, 1.0)
    P.close()
