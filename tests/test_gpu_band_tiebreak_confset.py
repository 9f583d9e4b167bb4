"""GPU parity of the lower validation bound (Remark 2, two-sided bands), randomised calibration
(the adjoined uniform of Section 7.1) and confidence sets from calibration (Section 8) through
the C ABI vs the oracle.

Bars: rejection counts, k, the tie-break thresholds c_i (uint32), counts below the pair
threshold and keep masks bit-exact; lambda_i exact (float32 keys, or the float64 statistic
table of the 2-arm design); Clopper-Pearson lower bounds and lower Tilt-Bounds within 1e-9
relative or 1e-13 absolute (the GPU takes cp_lower = 1 - cp_upper(N - R), the oracle
Beta^{-1}(delta; R, N - R + 1) directly); estimand ranges within 1e-12.
Inputs that are arguments of an entry point (rejection counts R, thresholds lambda, observed
statistics s) are seeded synthetic values where no simulation is involved.
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


def _dev(a, dtype=torch.float64):
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def _case(design):
    if design == "ztest1":
        return W.ztest_1d(40, 3000)
    if design == "binom2":
        return W.binom2_grid(12, 3000, lo=-2.0, hi=0.5, seed=1)
    if design == "hier4":
        return W.hier4_grid(2, 3000, seed=1)
    if design == "basket4":
        return W.basket_grid(2, 3000, lo=-2.4, hi=-0.9, seed=1)
    return W.phase23_grid((2, 2, 1, 1), 300, seed=1)


def _oracle_lower(design, w, subs, R, delta):
    box = np.array([s[0] for s in subs])
    N = w["sims"][box]
    cpl = O.cp_lower(R, N, delta)
    lb, _ = O.tile_lower(O.family_of(design), w["theta"][box], O._pad_vertices(subs, w["theta"]), cpl,
                         n=O.n_of(design))
    return cpl, lb


# ------------------------------------------------------------------ lower bound / band
def test_lower_band_binom2_end_to_end():
    w = W.binom2_grid(16, 2000, lo=-2.0, hi=0.5, seed=2)
    print("[band] binom2 end to end", flush=True)
    P = cse.Platten.create("binom2", w["theta"], w["radii"], w["sims"])
    v = P.validate(seed=2, delta=0.01)
    lo = P.validate_lower(v["reject"], delta=0.01)
    torch.cuda.synchronize()
    ov = O.validate("binom2", w["theta"], w["radii"], w["sims"], 2, 0.01)
    assert np.array_equal(_np(v["reject"]), ov["R"])
    np.testing.assert_allclose(_np(lo["cp_lower"]), ov["cp_lower"], rtol=1e-9, atol=1e-13)
    np.testing.assert_allclose(_np(lo["lower"]), ov["lower"], rtol=1e-9, atol=1e-13)
    # a band: lower <= cp_lower <= R / N <= cp_upper <= upper
    f = ov["R"] / ov["N"]
    assert np.all(_np(lo["lower"]) <= _np(lo["cp_lower"]) + 1e-15)
    assert np.all(_np(lo["cp_lower"]) <= f + 1e-15) and np.all(f <= _np(v["cp_upper"]) + 1e-15)
    assert np.all(_np(v["cp_upper"]) <= _np(v["tile_bound"]) + 1e-15)
    P.close()


@pytest.mark.parametrize("design", ["ztest1", "hier4", "phase23"])
def test_lower_synthetic_counts(design):
    w = _case(design)
    P = cse.Platten.create(design, w["theta"], w["radii"], w["sims"], cut=w.get("cut"))
    subs = O.subtiles(design, w["theta"], w["radii"])
    box = np.array([s[0] for s in subs])
    N = w["sims"][box]
    rng = np.random.default_rng(7)
    R = (rng.uniform(0, 1, len(subs)) ** 3 * N).astype(np.int32)
    R[0], R[-1] = 0, N[-1]                     # the two ends: cp_lower = 0 and cp_lower = delta^(1/N)
    print(f"[band] {design}: {len(subs)} tiles, synthetic counts", flush=True)
    lo = P.validate_lower(_dev(R, torch.int32), delta=0.05)
    torch.cuda.synchronize()
    cpl, lb = _oracle_lower(design, w, subs, R, 0.05)
    np.testing.assert_allclose(_np(lo["cp_lower"]), cpl, rtol=1e-9, atol=1e-13)
    np.testing.assert_allclose(_np(lo["lower"]), lb, rtol=1e-9, atol=1e-13)
    assert _np(lo["lower"])[0] == 0.0 and _np(lo["cp_lower"])[0] == 0.0
    P.close()


# ------------------------------------------------------------------ randomised calibration
def _tiebreak_compare(design, w, seed, alpha=0.05):
    print(f"[tiebreak] {design} {w['name']} seed={seed}", flush=True)
    P = cse.Platten.create(design, w["theta"], w["radii"], w["sims"], cut=w.get("cut"))
    g = P.calibrate_tiebreak(seed, alpha=alpha)
    plain = P.calibrate(seed, alpha=alpha, with_validation=False)
    torch.cuda.synchronize()
    key = np.float64 if design == "binom2" else np.float32
    cut = w.get("cut", 1.96) if design != "hier4" else 0.05
    oc = O.calibrate_tiebreak(design, w["theta"], w["radii"], w["sims"], seed, alpha, key_dtype=key, cut=cut)
    k = _np(g["k"])
    ap = oc["alpha_prime"]
    frac = (oc["N"] + 1.0) * ap
    near = np.abs(frac - np.round(frac)) < 1e-7
    assert np.all((k == oc["k"]) | near)
    same = k == oc["k"]
    assert same.mean() > 0.9
    lam = _np(g["lambda_tile"])
    u = _np(g["u_tile"]).view(np.uint32)
    if design == "ztest1":
        # X is drawn in float32 on the GPU and in float64 by the oracle: lambda agrees to 2e-6,
        # and c must be the uniform of a simulation whose statistic is within that of lambda
        np.testing.assert_allclose(lam, oc["lam"], rtol=0, atol=2e-6)
        _, _, S = O._tile_simulation(design, w["theta"], w["sims"], oc["subs"], seed, 1.96, True)
        uu = O.tiebreak_u(seed, int(oc["N"].max()))
        for t in range(len(lam)):
            near = np.flatnonzero(np.abs(S[t, : oc["N"][t]] - lam[t]) <= 2e-6)
            assert int(u[t]) in set(uu[near].tolist())
        assert np.mean(u.astype(np.int64) == oc["c"]) >= 0.9
        assert np.array_equal(_np(g["reject_at_lambda"]), np.maximum(k - 1, 0))
        P.close()
        return oc
    assert np.array_equal(lam[same], oc["lam"][same])
    assert np.array_equal(u[same].astype(np.int64), oc["c"][same])
    assert np.array_equal(_np(g["reject_at_lambda"])[same], oc["reject_at"][same])
    # the plain calibration's threshold is the first component of the pair
    assert np.array_equal(_np(plain["lambda_tile"]), lam)
    assert np.all(_np(g["reject_at_lambda"]) >= _np(plain["reject_at_lambda"]))
    if same.all():
        assert float(_np(g["lambda_global"])[0]) == oc["lam_global"]
        assert int(_np(g["u_global"]).view(np.uint32)[0]) == oc["c_global"]
    P.close()
    return oc


@pytest.mark.parametrize("design", ["ztest1", "binom2", "hier4", "phase23", "basket4"])
def test_tiebreak_parity(design):
    oc = _tiebreak_compare(design, _case(design), seed=5)
    assert np.all(oc["reject_at"] == np.maximum(oc["k"] - 1, 0))


def test_tiebreak_many_ties_radix_fallback():
    """A tile whose tie class at lambda holds more than 4,096 simulations: more than the 2-arm
    batch tie-break's 256-word first-pass region, so one 8-bit histogram pass and a gather pass
    pick c."""
    w = dict(name="binom2_ties", theta=np.array([[-4.0, -4.0], [-1.0, -1.2]]), radii=np.full((2, 2), 0.05),
             sims=np.array([100_000, 5000], np.int32))
    oc = _tiebreak_compare("binom2", w, seed=3, alpha=0.025)
    _, _, S = O._tile_simulation("binom2", w["theta"], w["sims"], oc["subs"], 3, 1.96, True)
    ties = [int(np.sum(S[t, : oc["N"][t]] == oc["lam"][t])) for t in range(len(oc["subs"]))]
    print(f"[tiebreak] tie class sizes {ties}", flush=True)
    assert max(ties) > 4096


def test_tiebreak_heavy_ties_two_histogram_passes():
    """Tie classes of about 200,000 simulations in one batch (theta near (-5, -5), alpha 0.3:
    lambda is the statistic of the equal-count outcomes): the 2-arm batch tie-break overflows its
    first-pass regions and needs two 8-bit histogram passes before the candidate bins fit LDS."""
    w = dict(name="binom2_heavy_ties", theta=np.array([[-5.0, -5.0], [-4.8, -5.0], [-1.0, -1.2]]),
             radii=np.full((3, 2), 0.05), sims=np.full(3, 300_000, np.int32))
    oc = _tiebreak_compare("binom2", w, seed=3, alpha=0.3)
    _, _, S = O._tile_simulation("binom2", w["theta"], w["sims"], oc["subs"], 3, 1.96, True)
    ties = [int(np.sum(S[t, : oc["N"][t]] == oc["lam"][t])) for t in range(len(oc["subs"]))]
    print(f"[tiebreak] tie class sizes {ties}", flush=True)
    assert max(ties) > 512 * 256


def test_tiebreak_global_pair_many_tiles():
    """More than 65,536 tiles (the global pair is reduced by partial minima, then one workgroup):
    (lambda*, c*) is the lexicographic minimum of the per-tile pairs over the null-space tiles."""
    w = W.binom2_grid(300, 512, lo=-2.0, hi=0.5, lower_triangle=False, seed=4)
    P = cse.Platten.create("binom2", w["theta"], w["radii"], w["sims"], keep_all=True)
    assert P.n_tiles > 65_536
    print(f"[tiebreak] global pair over {P.n_tiles} tiles", flush=True)
    g = P.calibrate_tiebreak(4, alpha=0.05)
    torch.cuda.synchronize()
    lam = _np(g["lambda_tile"])
    u = _np(g["u_tile"]).view(np.uint32).astype(np.int64)
    inn = np.asarray(P.tiles["in_null"]).astype(bool)
    assert inn.any() and not inn.all()
    order = np.lexsort((u[inn], lam[inn]))
    assert float(_np(g["lambda_global"])[0]) == lam[inn][order[0]]
    assert int(_np(g["u_global"]).view(np.uint32)[0]) == u[inn][order[0]]
    P.close()


# ------------------------------------------------------------------ confidence sets
def test_confidence_set_ztest_classical():
    r = 0.0125
    theta = np.arange(-2.0 + r, 3.0, 2 * r)[:, None]
    w = dict(theta=theta, radii=np.full_like(theta, r), sims=np.full(len(theta), 20000, np.int32))
    print(f"[confset] ztest1 {len(theta)} tiles", flush=True)
    P = cse.Platten.create("ztest1", w["theta"], w["radii"], w["sims"], keep_all=True)
    g = P.calibrate(4, alpha=0.05, with_validation=False)
    oc = O.calibrate("ztest1", w["theta"], w["radii"], w["sims"], 4, 0.05, keep_all=True)
    torch.cuda.synchronize()
    # float32 draws on the GPU, float64 in the oracle: the thresholds agree to 2e-6; the set is
    # compared on the oracle's thresholds (an input of the entry point), and the classical
    # bound is checked on the GPU's own
    np.testing.assert_allclose(_np(g["lambda_tile"]), oc["lam"], rtol=0, atol=2e-6)
    lam_o = _dev(oc["lam"])
    for x in (0.7, 1.3, 2.2):
        own = P.confidence_set(-x, g["lambda_tile"], [1.0, 0.0])
        c = P.confidence_set(-x, lam_o, [1.0, 0.0])
        torch.cuda.synchronize()
        assert x - 1.6449 - 0.12 <= _np(own["e_range"])[0] <= x - 1.6449 + 0.04
        keep, lo, hi, rng = O.confidence_set(oc["subs"], oc["lam"], -x, [1.0, 0.0])
        assert np.array_equal(_np(c["keep"]).astype(bool), keep)
        np.testing.assert_allclose(_np(c["e_lo"]), lo, rtol=0, atol=1e-12)
        np.testing.assert_allclose(_np(c["e_hi"]), hi, rtol=0, atol=1e-12)
        np.testing.assert_allclose(_np(c["e_range"]), rng, rtol=0, atol=1e-12)
        assert x - 1.6449 - 0.12 <= _np(c["e_range"])[0] <= x - 1.6449 + 0.04
    P.close()


@pytest.mark.parametrize("link", ["linear", "expit"])
def test_confidence_set_binom2_per_tile_statistic(link):
    w = W.binom2_grid(10, 800, lo=-1.5, hi=0.5, lower_triangle=False, seed=3)
    P = cse.Platten.create("binom2", w["theta"], w["radii"], w["sims"], keep_all=True)
    oc = O.calibrate("binom2", w["theta"], w["radii"], w["sims"], 3, 0.05, keep_all=True)
    subs = oc["subs"]
    assert any(len(s[2]) == 3 for s in subs)
    rng = np.random.default_rng(11)
    lam = oc["lam"]
    s = lam + rng.normal(0.0, 0.5, len(lam))
    s[::7] = lam[::7]                                   # equal to the threshold: kept
    coef = np.array([-1.0, 1.0, 0.1])
    print(f"[confset] binom2 {len(subs)} tiles, link {link}", flush=True)
    c = P.confidence_set(_dev(s), _dev(lam), coef, link=link)
    torch.cuda.synchronize()
    keep, lo, hi, rr = O.confidence_set(subs, lam, s, coef, link, key_dtype=np.float64)
    assert 0 < keep.sum() < len(keep)
    assert np.array_equal(_np(c["keep"]).astype(bool), keep)
    np.testing.assert_allclose(_np(c["e_lo"]), lo, rtol=0, atol=1e-12)
    np.testing.assert_allclose(_np(c["e_hi"]), hi, rtol=0, atol=1e-12)
    np.testing.assert_allclose(_np(c["e_range"]), rr, rtol=0, atol=1e-12)
    P.close()


@pytest.mark.parametrize("design", ["hier4", "phase23"])
def test_confidence_set_4d_float32_compare(design):
    w = _case(design)
    P = cse.Platten.create(design, w["theta"], w["radii"], w["sims"], cut=w.get("cut"))
    subs = O.subtiles(design, w["theta"], w["radii"])
    n = len(subs)
    rng = np.random.default_rng(12)
    lam = rng.uniform(0.0, 0.2, n).astype(np.float32).astype(np.float64)
    lam[0], lam[1] = -np.inf, np.inf
    s = lam + rng.normal(0.0, 0.05, n)
    s[2::5] = lam[2::5] - 1e-12                          # below in float64, equal in float32: kept
    s[0], s[1] = -1.0, 1.0
    coef = np.array([-3.0, 1.0, 1.0, 1.0, 0.0])
    print(f"[confset] {design}: {n} tiles", flush=True)
    for link in ("linear", "expit"):
        c = P.confidence_set(_dev(s), _dev(lam), coef, link=link)
        torch.cuda.synchronize()
        keep, lo, hi, rr = O.confidence_set(subs, lam, s, coef, link)
        assert keep[0] and not keep[1]
        assert np.array_equal(_np(c["keep"]).astype(bool), keep)
        np.testing.assert_allclose(_np(c["e_lo"]), lo, rtol=0, atol=1e-12)
        np.testing.assert_allclose(_np(c["e_hi"]), hi, rtol=0, atol=1e-12)
        np.testing.assert_allclose(_np(c["e_range"]), rr, rtol=0, atol=1e-12)
    # nothing kept: the empty range
    c = P.confidence_set(10.0, _dev(np.full(n, np.inf)), coef)
    torch.cuda.synchronize()
    assert _np(c["keep"]).sum() == 0
    assert tuple(_np(c["e_range"])) == (np.inf, -np.inf)
    with pytest.raises(cse.CseError):
        cse.cse_confidence_set(P.handle, _dev([0.0]), 0, _dev(lam), coef, 2, c["keep"], c["e_lo"], c["e_hi"],
                               c["e_range"])
    P.close()


def test_full_c2_workload_sampled_boxes():
    """The headline 2-arm workload (256 x 256 boxes kept to theta1 <= theta0, 8,192 sims):
    randomised calibration, the lower bound and a confidence set over all 32,896 tiles in one
    launch each, compared with the oracle on sampled boxes (a diagonal one among them)."""
    w = W.binom2_256_tri()
    th, rd, sm = w["theta"], w["radii"], w["sims"]
    P = cse.Platten.create("binom2", th, rd, sm)
    print(f"[full c2] {P.n_tiles} tiles", flush=True)
    g = P.calibrate_tiebreak(w["seed"], alpha=w["alpha"])
    v = P.validate(w["seed"], delta=w["delta"])
    lo = P.validate_lower(v["reject"], delta=w["delta"])
    coef = np.array([-1.0, 1.0, 0.0])
    c = P.confidence_set(_dev(np.zeros(P.n_tiles)), g["lambda_tile"], coef)
    torch.cuda.synchronize()
    box = P.tiles["box"]
    rng = np.random.default_rng(3)
    diag = np.flatnonzero(np.isclose(th[:, 0], th[:, 1]))
    pick = np.unique(np.concatenate([[0, len(th) - 1], rng.choice(len(th), 3, replace=False), diag[:1]]))
    sub = W.subsample(w, pick)
    oc = O.calibrate_tiebreak("binom2", sub["theta"], sub["radii"], sub["sims"], w["seed"], w["alpha"])
    ov = O.validate("binom2", sub["theta"], sub["radii"], sub["sims"], w["seed"], w["delta"])
    ids = np.concatenate([np.flatnonzero(box == b) for b in pick])
    assert len(ids) == len(oc["lam"])
    assert 3 in P.tiles["n_vert"][ids]                            # the diagonal box is a triangle
    k = _np(g["k"])[ids]
    same = k == oc["k"]
    assert same.mean() >= 0.8
    assert np.array_equal(_np(g["lambda_tile"])[ids][same], oc["lam"][same])
    assert np.array_equal(_np(g["u_tile"]).view(np.uint32)[ids][same].astype(np.int64), oc["c"][same])
    assert np.array_equal(_np(g["reject_at_lambda"])[ids][same], oc["reject_at"][same])
    assert np.array_equal(_np(v["reject"])[ids], ov["R"])
    np.testing.assert_allclose(_np(lo["lower"])[ids], ov["lower"], rtol=1e-9, atol=1e-13)
    keep, elo, ehi, _ = O.confidence_set(ov["subs"], oc["lam"], 0.0, coef, key_dtype=np.float64)
    assert np.array_equal(_np(c["keep"])[ids].astype(bool)[same], keep[same])
    np.testing.assert_allclose(_np(c["e_lo"])[ids], elo, rtol=0, atol=1e-12)
    P.close()
