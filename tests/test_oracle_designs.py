"""Pins of the oracle's designs, score gradient and calibration against exact results.

- pooled two-proportion z: z^2 equals Pearson's chi-square of the 2x2 table (scipy's
  chi2_contingency without continuity correction), sign from the difference;
- z-test Monte Carlo TIE and score gradient vs the closed forms 1 - Phi(1.96 - theta)
  and phi(1.96 - theta);
- 2-arm Monte Carlo TIE and score gradient vs exact enumeration over the 36 x 36 outcomes;
- common random numbers: counts are monotone in theta for a fixed simulation;
- calibration: Theorem 4 (f(lambda*) ~ Beta(k, N-k+1) for a continuous statistic, KS test
  over 200 seeds) and the shift invariant lambda*_i + theta_i = const under CRN (z-test).
"""
import math

import numpy as np
import pytest
from scipy import stats

import oracle as O

N35 = 35


def test_pooled_z_equals_pearson_chi_square():
    for y0 in range(0, 36, 3):
        for y1 in range(0, 36, 2):
            z = O.pooled_z(y0, y1)
            tab = np.array([[y0, N35 - y0], [y1, N35 - y1]])
            if y0 + y1 in (0, 2 * N35):
                assert z == 0.0
                continue
            chi2 = stats.chi2_contingency(tab, correction=False)[0]
            assert z * z == pytest.approx(chi2, rel=1e-12, abs=1e-12)
            assert np.sign(z) == np.sign(y1 - y0)


def test_ztest_tie_and_gradient_closed_form():
    th = -1 + (2 * np.arange(64) + 1) / 128
    N = 10_000
    R, sz, _ = O.sim_ztest1(th, np.full(64, N, np.int32), seed=0)
    f = stats.norm.sf(1.96 - th)
    se = np.sqrt(f * (1 - f) / N)
    assert np.all(np.abs(R / N - f) < 5 * se)
    g = O.score_gradient("ztest1", th[:, None], R, sz, np.full(64, N))[:, 0]
    gexact = stats.norm.pdf(1.96 - th)
    # per-simulation variance of reject*Z is bounded by E[Z^2 1{rej}] <= 4 f for these tiles
    assert np.all(np.abs(g - gexact) < 5 * np.sqrt(8 * f / N))


def _exact_binom2(theta, cut=1.96, n=N35):
    p = 1.0 / (1.0 + np.exp(-np.asarray(theta, float)))
    y = np.arange(n + 1)
    pm = np.outer(stats.binom.pmf(y, n, p[0]), stats.binom.pmf(y, n, p[1]))
    rej = np.array([[O.pooled_z(a, b, n) > cut for b in y] for a in y], float)
    f = float(np.sum(pm * rej))
    g0 = float(np.sum(pm * rej * (y[:, None] - n * p[0])))
    g1 = float(np.sum(pm * rej * (y[None, :] - n * p[1])))
    return f, np.array([g0, g1])


@pytest.mark.parametrize("theta", [(0.0, 0.0), (-1.0, -1.0), (-3.0, -3.0), (-0.5, -0.6), (0.6, 0.1)])
def test_binom2_mc_vs_exact_enumeration(theta):
    N = 20_000
    R, sT, _ = O.sim_binom2(np.array([theta]), np.array([N], np.int32), seed=1)
    f, g = _exact_binom2(theta)
    assert abs(R[0] / N - f) < 5 * math.sqrt(f * (1 - f) / N)
    ghat = O.score_gradient("binom2", np.array([theta]), R, sT, np.array([N]))[0]
    # per-sim score term reject*(y - n p) has |.| <= 35: bound its variance by 35^2 f
    assert np.all(np.abs(ghat - g) < 5 * math.sqrt(N35**2 * f / N))


def test_binom2_exact_values_symmetry():
    """At theta0 = theta1 the gradient components are opposite (the test is antisymmetric
    under swapping the arms together with the sign of z)."""
    f, g = _exact_binom2((0.0, 0.0))
    assert g[0] == pytest.approx(-g[1], rel=1e-12)
    assert 0.0 < f < 0.025


def test_crn_counts_monotone_in_theta():
    th = np.linspace(-2, 1, 13)
    Ys = np.stack([O.arm_counts([t, t], 200, seed=4) for t in th])  # [13, 200, 2]
    assert np.all(np.diff(Ys, axis=0) >= 0)


def test_binom2_sumT_is_sum_over_rejections():
    th = np.array([[0.2, 0.5]])
    N = 500
    R, sT, S = O.sim_binom2(th, np.array([N], np.int32), seed=2, want_S=True)
    Y = O.arm_counts(th[0], N, seed=2)
    rej = -S[0] > 1.96
    assert R[0] == rej.sum()
    assert np.array_equal(sT[0], Y[rej].sum(axis=0))


def test_calibration_theorem4_beta_law():
    """f(lambda*) ~ Beta(k, N-k+1) for i.i.d. continuous S (Theorem 4 proof)."""
    N, k, th = 999, 25, -0.3
    vals = []
    for seed in range(200):
        _, _, S = O.sim_ztest1(np.array([th]), np.array([N], np.int32), seed=seed + 100, want_S=True)
        lam = O.order_statistic(S[0], k)
        vals.append(stats.norm.sf(-lam - th))      # P(S < lam) = P(X > -lam)
    vals = np.array(vals)
    assert stats.kstest(vals, stats.beta(k, N - k + 1).cdf).pvalue > 1e-3
    assert abs(vals.mean() - k / (N + 1)) < 5 * stats.beta(k, N - k + 1).std() / math.sqrt(200)


def test_calibration_ztest_shift_invariant():
    th = -1 + (2 * np.arange(64) + 1) / 128
    out = O.calibrate("ztest1", th[:, None], np.full((64, 1), 1 / 128), np.full(64, 2000, np.int32),
                      seed=0, alpha=0.025)
    assert np.all(out["k"] == out["k"][0])
    s = out["lam"] + th
    assert np.ptp(s) < 1e-12
    assert out["lam_global"] == out["lam"][np.argmax(th)]
    assert np.all(out["reject_at_lam"] == out["k"] - 1)      # continuous S: exactly k-1 below S_(k)


def test_order_statistic_k_zero():
    assert O.order_statistic(np.array([0.3, 0.1]), 0) == -math.inf
    assert O.order_statistic(np.array([0.3, 0.1, 0.2]), 2) == 0.2
