"""Pins of the oracle's basket design (Section 10.1's validation case study; Berry et al.'s
basket trial: four arms against fixed rates p_0a, 85% posterior rule), each against something
other than the oracle's own arithmetic:

- the posterior tail P(p_a > p_0a | y) against direct numerical integration of the exact
  posterior (sigma^2 on a log grid, mu on a grid, each arm's offset integrated on a grid that
  contains 0): the Laplace node mixture converges to it as n grows (within 0.01 at n = 2000,
  also with unequal p_0a), and is within 0.05 at n = 35;
- exchangeability: permuting the arms (counts and p_0a together) permutes the statistics;
- the pieces box ∩ P(b) partition each box, and a sampled point's null configuration is its
  piece's b;
- the design simulation replayed from the pinned arm counts, the pinned posterior and the
  85% rule.
"""
import itertools

import numpy as np
import pytest
from scipy import special, stats

import oracle as O


def _exact_tail(y, n, theta0, ns2=150):
    """P(theta_a > theta_0a | y) for the hierarchical model on the offsets, by quadrature."""
    y = np.asarray(y)
    theta0 = np.asarray(theta0, np.float64)
    dhat = np.log((y + 0.5) / (n - y + 0.5)) - theta0
    sd_lik = 1.0 / np.sqrt(n * 0.25 * (1 - np.abs(2 * (y + 0.5) / (n + 1) - 1)) + 1.0)
    ls2 = np.linspace(np.log(1e-6), np.log(1e3), ns2)
    s2 = np.exp(ls2)
    w_s2 = np.full(ns2, ls2[1] - ls2[0])
    w_s2[[0, -1]] *= 0.5
    a_, b_ = 0.0005, 0.000005
    logp_s2 = a_ * np.log(b_) - special.gammaln(a_) - (a_ + 1) * ls2 - b_ / s2 + ls2 + np.log(w_s2)
    c = dhat.mean()
    mu = np.unique(np.concatenate([np.linspace(-8, 6, 141), np.linspace(c - 1.5, c + 1.5, 601)]))
    w_mu = np.zeros(len(mu))
    dm = np.diff(mu)
    w_mu[:-1] += dm / 2
    w_mu[1:] += dm / 2
    logp_mu = stats.norm.logpdf(mu, -1.34, 10.0) + np.log(w_mu)
    gh_x, gh_w = np.polynomial.hermite_e.hermegauss(40)
    gh_w = gh_w / np.sqrt(2 * np.pi)
    logL = np.zeros((ns2, len(mu)))
    tails = np.zeros((4, ns2, len(mu)))
    for a in range(4):
        h = sd_lik[a] / 12.0
        lo, hi = int(np.floor((dhat[a] - 12 * sd_lik[a]) / h)), int(np.ceil((dhat[a] + 12 * sd_lik[a]) / h))
        lo, hi = min(lo, -1), max(hi, 1)
        d = h * np.arange(lo, hi + 1)                       # contains 0
        tw = np.full(len(d), h)
        tw[[0, -1]] *= 0.5
        tpos = np.where(d > 0, h, 0.0)
        tpos[d == 0] = 0.5 * h
        tpos[-1] *= 0.5
        lik = np.exp(stats.binom.logpmf(y[a], n, special.expit(d + theta0[a])))
        for i in range(ns2):
            sd = np.sqrt(s2[i])
            if sd < 2 * h:        # the normal is narrow against the likelihood: Gauss-Hermite
                x = mu[:, None] + sd * gh_x[None, :]
                lk = np.exp(stats.binom.logpmf(y[a], n, special.expit(x + theta0[a])))
                m = (lk * gh_w).sum(1)
                t = (lk * gh_w * (x > 0)).sum(1)
            else:
                lk = lik[None, :] * stats.norm.pdf(d[None, :], mu[:, None], sd)
                m = (lk * tw).sum(1)
                t = (lk * tpos).sum(1)
            logL[i] += np.log(np.maximum(m, 1e-300))
            tails[a, i] = t / np.maximum(m, 1e-300)
    lw = logL + logp_s2[:, None] + logp_mu[None, :]
    w = np.exp(lw - lw.max())
    w /= w.sum()
    return np.array([(w * tails[a]).sum() for a in range(4)])


@pytest.mark.parametrize("y,n,theta0,tol", [
    ([300, 380, 250, 440], 2000, None, 0.01),
    ([310, 290, 330, 300], 2000, None, 0.01),
    ([100, 40, 70, 150], 400, [-1.0, -2.0, -1.5, -0.5], 0.01),
    ([2, 5, 9, 14], 35, None, 0.05),
])
def test_posterior_tail_vs_quadrature(y, n, theta0, tol):
    t0 = O.BASKET_THETA0 if theta0 is None else np.asarray(theta0)
    ex = _exact_tail(y, n, t0)
    lap = 1.0 - O.basket_complement(y, n, t0)
    print(y, n, np.round(ex, 5), np.round(lap, 5))
    assert np.max(np.abs(ex - lap)) < tol


def test_exchangeability():
    t0 = np.array([-1.0, -2.0, -1.5, -0.5])
    y = np.array([7, 3, 12, 20])
    base = O.basket_complement(y, 35, t0)
    for perm in itertools.permutations(range(4)):
        p = list(perm)
        np.testing.assert_allclose(O.basket_complement(y[p], 35, t0[p]), base[p], rtol=1e-9, atol=1e-15)
    eq = O.basket_complement([6, 6, 6, 6])
    assert np.ptp(eq) < 1e-12


def test_monotone_in_own_count():
    prev = None
    for k in range(2, 30):
        s = O.basket_complement([k, 6, 9, 4])
        if prev is not None:
            assert s[0] < prev
        prev = s[0]


@pytest.mark.parametrize("seed", [0, 1])
def test_pieces_partition_the_box(seed):
    rng = np.random.default_rng(seed)
    t0 = np.array([-1.7, -1.0, -2.0, -0.5])
    theta = t0 + rng.uniform(-0.2, 0.2, (6, 4))
    radii = rng.uniform(0.05, 0.3, (6, 4))
    pieces = O.basket_subboxes(theta, radii, t0)
    for i in range(6):
        mine = [p for p in pieces if p[0] == i]
        assert [p[1] for p in mine] == sorted(p[1] for p in mine)
        x = theta[i] + rng.uniform(-1, 1, (4000, 4)) * radii[i]
        b_true = ((x <= t0) * (1 << np.arange(4))).sum(1)
        hit = np.zeros(len(x), int)
        for _, b, c, r in mine:
            inside = np.all(np.abs(x - c) <= r, axis=1)
            assert np.all(b_true[inside] == b)
            hit += inside
        assert np.all(hit[b_true > 0] == 1) and np.all(hit[b_true == 0] == 0)
        vol = sum(np.prod(2 * r) for _, _, _, r in mine)
        assert vol == pytest.approx(np.prod(2 * radii[i]) * np.mean(b_true > 0), abs=0.05 * np.prod(2 * radii[i]))


def test_simulation_replay():
    t0 = O.BASKET_THETA0
    centres = np.array([[-1.8, -1.6, -2.2, -1.0], [-1.0, -1.9, -1.8, -1.75]])
    cfg = np.array([0b0101, 0b1110], np.int32)
    sims = np.array([60, 60], np.int32)
    R, sT, S = O.sim_basket(centres, cfg, sims, seed=3, want_S=True)
    for t in range(2):
        Y = O.arm_counts(centres[t], 60, 3)
        r, st = 0, np.zeros(4, np.int64)
        for k in range(60):
            sc = O.basket_complement(Y[k], 35, t0)
            s = min(sc[a] for a in range(4) if (cfg[t] >> a) & 1)
            assert S[t, k] == s
            if s < O.BASKET_CUT:
                r += 1
                st += Y[k]
        assert R[t] == r and np.array_equal(sT[t], st)
    assert R.sum() > 0
