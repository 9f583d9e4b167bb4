"""Pins of the oracle's random stream and draw rules against external facts.

- Philox4x32-10 against the published known-answer values (tests/golden/philox_kat.txt).
- The stream layout word(seed, k, w) against the block function.
- The Bernoulli threshold rule at its exact special points, and the law of
  the counts it produces (chi-square against Binomial(35, p)).
- Box-Muller normals against the standard normal law (KS).
"""
import math

import numpy as np
import pytest
from scipy import stats

import oracle as O
from conftest import read_golden


def test_philox_known_answers():
    rows = read_golden("philox_kat.txt")
    assert len(rows) == 3
    for r in rows:
        v = [int(x, 16) for x in r]
        out = O.philox(v[0:4], v[4:6])
        assert [int(x) for x in out] == v[6:10]


def test_word_layout_matches_block_function():
    seed = (7 << 32) | 12345
    for k in (0, 1, 77, 2**31 + 5):
        for w in (0, 1, 2, 3, 4, 69, 139):
            blk = O.philox([w // 4, k, 0, 0], [seed & 0xFFFFFFFF, seed >> 32])
            assert O.word(seed, k, w) == int(blk[w % 4])


def test_threshold_special_points():
    assert O.bern_threshold(0.0) == 2**31                     # expit(0) = 1/2 exactly
    assert O.bern_threshold(800.0) == 2**32 - 1                # clamped top
    assert O.bern_threshold(-800.0) == 0
    # monotone in theta
    th = np.linspace(-6, 6, 2001)
    T = np.array([O.bern_threshold(t) for t in th])
    assert np.all(np.diff(T.astype(np.int64)) >= 0)
    # within one unit of 2^32 expit(theta)
    for t in (-3.0, -1.0 + 1 / 128, 0.4925, 1.1527):
        exact = 2.0**32 / (1.0 + math.exp(-t))
        assert abs(O.bern_threshold(t) - exact) <= 0.5 + 1e-6


def test_uniform_words_chi_square():
    w = np.array([O.word(3, k, j) for k in range(4096) for j in range(8)], np.uint64)
    counts = np.bincount((w >> 24).astype(np.int64), minlength=256)
    p = stats.chisquare(counts).pvalue
    assert p > 1e-4


@pytest.mark.parametrize("theta", [-2.0, 0.3, 1.0])
def test_binomial_counts_law(theta):
    n = 35
    Y = O.arm_counts([theta, -theta], 20000, seed=11, n=n)
    p = 1.0 / (1.0 + math.exp(-theta))
    for a, pa in ((0, p), (1, 1 - p)):
        obs = np.bincount(Y[:, a], minlength=n + 1).astype(float)
        exp = stats.binom.pmf(np.arange(n + 1), n, pa) * Y.shape[0]
        # pool sparse cells so the chi-square approximation holds
        keep = exp >= 5
        o = np.concatenate([obs[keep], [obs[~keep].sum()]])
        e = np.concatenate([exp[keep], [exp[~keep].sum()]])
        if e[-1] == 0:
            o, e = o[:-1], e[:-1]
        stat = ((o - e) ** 2 / e).sum()
        assert stats.chi2.sf(stat, len(o) - 1) > 1e-4
    # the two arms use disjoint words: independent counts
    r = np.corrcoef(Y[:, 0], Y[:, 1])[0, 1]
    assert abs(r) < 5.0 / math.sqrt(Y.shape[0])


def test_box_muller_normal_law():
    z = np.array([O.lib().orc_box_muller(O.word(5, k, 0), O.word(5, k, 1)) for k in range(20000)])
    assert stats.kstest(z, "norm").pvalue > 1e-4
    assert abs(z.mean()) < 5 / math.sqrt(z.size)
    assert abs(z.var() - 1.0) < 5 * math.sqrt(2.0 / z.size)
