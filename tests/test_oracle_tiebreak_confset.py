"""Pins of the oracle's randomised calibration (the adjoined uniform of the discussion of
Theorem (pointwise calibration), Section 7.1) and of confidence sets from calibration
(Section 8), each against something other than the oracle's own formulas:

- the tie-break stream against the Philox block function (pinned by published known-answer
  values) and a uniformity check; the pair order statistic against Python's tuple sort;
- Theorem (pointwise calibration) on a discrete statistic: with exact rejection probabilities
  from full enumeration of the 2-arm outcomes, the mean of f(lambda_hat) over independent
  calibrations sits at floor((N+1) alpha)/(N+1) for the randomised test, and inside the
  theorem's interval [.. - E Delta f, ..] without the tie-break;
- z-test confidence bound against the classical X - z_{1-alpha}, and exact conditional
  coverage Phi(...) of every tile's test;
- the image of each tile under e against e at dense points of the tile.
"""
import numpy as np
import pytest
from scipy import stats

import oracle as O

N35 = 35


def test_tiebreak_stream_is_the_philox_block_and_uniform():
    u = O.tiebreak_u(123456789, 5000)
    for k in (0, 1, 77, 4999):
        assert u[k] == O.philox([0, k, 1, 0], [123456789 & 0xFFFFFFFF, 123456789 >> 32])[0]
    # disjoint from the data words of the same simulation
    assert all(u[k] != O.word(123456789, k, 0) for k in range(50))
    x = (u.astype(np.float64) + 0.5) / 2.0 ** 32
    assert stats.kstest(x, "uniform").pvalue > 1e-4
    assert len(O.tiebreak_u(5, 0)) == 0


def test_pair_order_statistic_brute_force():
    rng = np.random.default_rng(3)
    S = rng.integers(0, 6, 300).astype(np.float64)     # heavy ties
    u = rng.integers(0, 2 ** 32, 300, dtype=np.uint64).astype(np.uint32)
    srt = sorted(zip(S.tolist(), u.tolist()))
    for k in (1, 2, 57, 150, 299, 300):
        assert O.order_statistic_pair(S, u, k) == (srt[k - 1][0], srt[k - 1][1])
    assert O.order_statistic_pair(S, u, 0) == (-np.inf, 0)


def _binom2_law(theta):
    """Exact law of S = -z over the 36 x 36 outcomes: (values, probabilities)."""
    y = np.arange(N35 + 1)
    p = 1.0 / (1.0 + np.exp(-np.asarray(theta, np.float64)))
    P = stats.binom.pmf(y, N35, p[0])[:, None] * stats.binom.pmf(y, N35, p[1])[None, :]
    S = np.array([[-O.pooled_z(a, b) for b in y] for a in y])
    return S.ravel(), P.ravel()


def test_pointwise_calibration_theorem_randomised_vs_plain():
    theta = np.array([-2.4, -2.4])           # small counts: a coarse, heavily tied statistic
    Sv, Pv = _binom2_law(theta)
    N, alpha = 99, 0.05
    k = int(np.floor((N + 1) * alpha))       # 5
    target = k / (N + 1)
    M = 2000
    f_rand = np.empty(M)
    f_plain = np.empty(M)
    jump = np.empty(M)
    for m in range(M):
        _, _, S = O.sim_binom2(theta[None, :], np.array([N], np.int32), seed=1000 + m, want_S=True)
        row = S[0, :N]
        u = O.tiebreak_u(1000 + m, N)
        lam, c = O.order_statistic_pair(row, u, k)
        below = Pv[Sv < lam].sum()
        at = Pv[Sv == lam].sum()
        f_rand[m] = below + at * (c / 2.0 ** 32)
        lam_plain = O.order_statistic(row, k)
        assert lam_plain == lam
        f_plain[m] = Pv[Sv < lam_plain].sum()
        jump[m] = Pv[Sv == lam_plain].sum()
    se = f_rand.std() / np.sqrt(M)
    # randomised: E f = floor((N+1) alpha)/(N+1) exactly (the statistic (S, u) is continuous)
    assert abs(f_rand.mean() - target) < 4.0 * se
    # plain: the theorem's interval, and a visible discreteness penalty at this point
    assert f_plain.mean() <= target + 4.0 * se
    assert f_plain.mean() >= target - jump.mean() - 4.0 * se
    assert target - f_plain.mean() > 5.0 * se


@pytest.mark.parametrize("design", ["ztest1", "binom2"])
def test_calibrate_tiebreak_consistent_with_plain(design):
    if design == "ztest1":
        theta = np.linspace(-0.9, -0.1, 5)[:, None]
        radii = np.full_like(theta, 0.1)
    else:
        theta = np.array([[-1.0, -1.0], [-2.0, -2.2], [-0.5, -0.7]])
        radii = np.full((3, 2), 0.1)
    sims = np.full(len(theta), 3000, np.int32)
    a = O.calibrate(design, theta, radii, sims, 9, 0.05)
    b = O.calibrate_tiebreak(design, theta, radii, sims, 9, 0.05)
    np.testing.assert_array_equal(a["lam"], b["lam"])
    np.testing.assert_array_equal(a["k"], b["k"])
    # distinct uniforms: exactly k - 1 pairs lie strictly below the k-th smallest
    np.testing.assert_array_equal(b["reject_at"], np.maximum(b["k"] - 1, 0))
    assert np.all(b["reject_at"] >= a["reject_at_lam"])
    g = int(np.argmin(a["lam"]))
    assert b["lam_global"] == a["lam_global"]
    tied = np.flatnonzero(b["lam"] == b["lam_global"])
    assert b["c_global"] == b["c"][tied].min()
    if design == "ztest1":
        assert g in tied


def _ztest_grid(lo=-2.0, hi=3.0, r=0.0125):
    theta = np.arange(lo + r, hi, 2 * r)[:, None]
    return theta, np.full_like(theta, r)


def test_ztest_confidence_bound_classical_and_coverage():
    theta, radii = _ztest_grid()
    sims = np.full(len(theta), 20000, np.int32)
    alpha = 0.05
    cal = O.calibrate("ztest1", theta, radii, sims, 4, alpha, keep_all=True)
    subs = cal["subs"]
    assert len(subs) == len(theta)                      # 0 is a box boundary: nothing clipped
    z = stats.norm.ppf(1 - alpha)
    for x in (0.7, 1.3, 2.2):
        keep, lo, hi, rng = O.confidence_set(subs, cal["lam"], -x, [1.0, 0.0])
        # S = -X rejects the tiles far below X: a lower confidence bound on theta
        assert x - z - 0.12 <= rng[0] <= x - z + 0.04
        assert rng[1] == pytest.approx(theta[-1, 0] + radii[-1, 0])
        # the kept tiles form one interval
        idx = np.flatnonzero(keep)
        assert np.array_equal(idx, np.arange(idx[0], len(theta)))
    # exact coverage of every tile's test at its worst point theta_i + r:
    # P(theta's tile kept) = P(-X >= lambda_i) = Phi(-lambda_i - theta)
    cov = stats.norm.cdf(-cal["lam"] - (theta[:, 0] + radii[:, 0]))
    assert cov.mean() >= 1 - alpha - 0.002
    assert cov.min() >= 1 - alpha - 0.006


@pytest.mark.parametrize("link", ["linear", "expit"])
def test_estimand_range_contains_tile_image(link):
    theta = np.array([[-0.5, -0.5], [0.3, -0.2], [-1.2, -1.6], [0.0, 0.4]])
    radii = np.full((4, 2), 0.15)
    subs = O.subtiles("binom2", theta, radii, keep_all=True)
    assert any(len(s[2]) == 3 for s in subs)
    coef = np.array([-1.0, 1.0, 0.25])                 # e = p1 - p0 + 1/4 (expit) or theta1 - theta0 + 1/4
    lo, hi = O.estimand_range(subs, coef, link)
    g = (lambda v: v) if link == "linear" else (lambda v: 1.0 / (1.0 + np.exp(-v)))
    rng = np.random.default_rng(5)
    for t, s in enumerate(subs):
        V = np.asarray(s[2])
        pts = np.vstack([V, rng.dirichlet(np.ones(len(V)), 400) @ V])
        e = g(pts) @ coef[:-1] + coef[-1]
        assert np.all(e >= lo[t] - 1e-12) and np.all(e <= hi[t] + 1e-12)
        if link == "linear" or len(V) == 4:            # exact: attained at a vertex
            ev = g(V) @ coef[:-1] + coef[-1]
            assert ev.min() == pytest.approx(lo[t], abs=1e-12)
            assert ev.max() == pytest.approx(hi[t], abs=1e-12)
    keep = np.zeros(len(subs), bool)
    keep[[0, 2]] = True
    lam = np.where(keep, -np.inf, np.inf)
    k2, lo2, hi2, rng2 = O.confidence_set(subs, lam, 0.0, coef, link)
    assert np.array_equal(k2, keep)
    assert rng2 == (min(lo[0], lo[2]), max(hi[0], hi[2]))
    _, _, _, empty = O.confidence_set(subs, np.full(len(subs), np.inf), 0.0, coef, link)
    assert empty == (np.inf, -np.inf)
