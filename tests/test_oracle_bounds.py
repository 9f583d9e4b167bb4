"""Pins of the oracle's bound arithmetic against the paper and against mathematics.

- worked values printed in the paper (2.73% bound, 0.23% gap; tests/golden/paper_tilt_values.txt);
- closed forms of the optimized normal Tilt-Bound and of its inverse (solving d/dq = 0 of
  the normal form of the bound by hand);
- the Renyi-divergence identity of Section 4.1 with D_q computed by brute-force summation
  over the binomial outcome space (checks the exponential-family psi and A);
- a dense brute-force q grid (checks the golden-section optimiser, Theorem 2);
- Theorem 1 itself with exact Type I Errors from enumeration (zero violations);
- vertices vs dense interior points (Theorem 3);
- Clopper-Pearson: closed forms at R = 0 and R = N - 1, and the defining tail identity
  P(Binom(N, u) <= R) = delta evaluated in 50-digit arithmetic (mpmath), not scipy.
"""
import itertools
import math

import mpmath as mp
import numpy as np
import pytest
from scipy import stats

import oracle as O
from conftest import read_golden

Z975 = stats.norm.ppf(0.975)


def f_z(theta):
    """Exact Type I Error of the one-sided z-test at level 2.5% (Section 4.3)."""
    return stats.norm.cdf(theta - Z975)


def test_paper_worked_values():
    rows = {r[0]: r for r in read_golden("paper_tilt_values.txt")}
    th0 = float(rows["optimized_bound"][1])
    v = float(rows["optimized_bound"][2])
    b, _ = O.tile_bound("normal", np.array([[th0]]), np.array([[[v]]]), np.array([f_z(th0)]))
    assert round(100 * b[0], int(rows["optimized_bound"][4])) == float(rows["optimized_bound"][3])
    # largest gap over target points theta0 + v, v in [0, 0.25], is at v = 0.25
    vs = np.linspace(0.0, 0.25, 101)
    bb, _ = O.tile_bound("normal", np.full((vs.size, 1), th0), vs[:, None, None],
                         np.full(vs.size, f_z(th0)))
    gap = bb - f_z(th0 + vs)
    assert np.argmax(gap) == vs.size - 1
    assert round(100 * gap.max(), int(rows["max_gap"][4])) == float(rows["max_gap"][3])


@pytest.mark.parametrize("a", [1e-4, 0.0137, 0.025, 0.2, 0.7])
@pytest.mark.parametrize("v", [1 / 512, 1 / 128, 0.05, 0.25, 1.0])
def test_normal_closed_forms(a, v):
    L = -math.log(a)
    closed = math.exp(-(math.sqrt(L) - v / math.sqrt(2)) ** 2) if math.sqrt(L) >= v / math.sqrt(2) else 1.0
    b, q = O.tile_bound("normal", np.array([[0.3]]), np.array([[[v], [-v]]]), np.array([a]))
    assert b[0] == pytest.approx(closed, rel=1e-10, abs=1e-14)
    if closed < 1.0:
        assert q[0] == pytest.approx(math.sqrt(2 * L) / v, rel=1e-5)
    closed_inv = math.exp(-(math.sqrt(L) + v / math.sqrt(2)) ** 2)
    ai, _ = O.tile_inverse("normal", np.array([[0.3]]), np.array([[[v], [-v]]]), a)
    assert ai[0] == pytest.approx(closed_inv, rel=1e-10)


def _binom_pmf2(theta, n=35):
    p = 1.0 / (1.0 + np.exp(-np.asarray(theta)))
    y = np.arange(n + 1)
    return np.outer(stats.binom.pmf(y, n, p[0]), stats.binom.pmf(y, n, p[1]))


def _binom_logpmf2(theta, n=35):
    p = 1.0 / (1.0 + np.exp(-np.asarray(theta)))
    y = np.arange(n + 1)
    return stats.binom.logpmf(y, n, p[0])[:, None] + stats.binom.logpmf(y, n, p[1])[None, :]


@pytest.mark.parametrize("theta0,v", [((0.0, 0.0), (0.1, -0.05)), ((-2.0, -2.5), (-0.3, 0.2)),
                                      ((1.0, -1.0), (0.01, 0.01))])
@pytest.mark.parametrize("q", [1.5, 4.0, 37.0])
def test_renyi_identity_bruteforce(theta0, v, q):
    """U = a^(1-1/q) exp{(1-1/q) D_q(P_{theta0+v} || P_theta0)} with D_q summed over outcomes."""
    from scipy.special import logsumexp
    lP = _binom_logpmf2(np.add(theta0, v))
    lQ = _binom_logpmf2(theta0)
    Dq = logsumexp(q * lP + (1 - q) * lQ) / (q - 1)
    a = 0.03
    lhs = O.log_tilt("binom", np.array(theta0), np.array(v), q, a)
    rhs = (1 - 1 / q) * math.log(a) + (1 - 1 / q) * Dq
    assert lhs == pytest.approx(rhs, rel=1e-9, abs=1e-12)


def test_golden_section_vs_dense_q_grid():
    rng = np.random.default_rng(0)
    m = 40
    th = rng.uniform(-3, 1, (m, 2))
    r = rng.choice([1 / 512, 1 / 128, 1 / 16, 0.25], m)
    V = np.array([[[sx * ri, sy * ri] for sx in (-1, 1) for sy in (-1, 1)] for ri in r])
    a = rng.uniform(0.001, 0.2, m)
    b, _ = O.tile_bound("binom", th, V, a)
    ai, _ = O.tile_inverse("binom", th, V, 0.025)
    ss = np.linspace(-12, 14, 6001)

    def grid_opt(fun, best):
        vals = np.array([fun(1.0 + math.exp(x)) for x in ss])
        j = int(best(vals))
        fine = np.linspace(ss[max(j - 2, 0)], ss[min(j + 2, ss.size - 1)], 4001)
        fv = np.array([fun(1.0 + math.exp(x)) for x in fine])
        return fv[best(fv)]

    for t in range(m):
        lu = grid_opt(lambda q: O.log_tilt("binom", th[t], V[t], q, a[t]).max(), np.argmin)
        li = grid_opt(lambda q: O.log_inv_tilt("binom", th[t], V[t], q, 0.025).min(), np.argmax)
        assert b[t] <= math.exp(lu) * (1 + 1e-12)
        assert b[t] >= math.exp(lu) * (1 - 1e-9)
        assert ai[t] >= math.exp(li) * (1 - 1e-12)
        assert ai[t] <= math.exp(li) * (1 + 1e-9)


def _exact_tie_binom2(theta, cut=1.96, n=35):
    y = np.arange(n + 1)
    rej = np.array([[O.pooled_z(a, b, n) > cut for b in y] for a in y])
    return float(np.sum(_binom_pmf2(theta, n) * rej))


def test_theorem1_holds_with_exact_tie():
    """Deterministic: inf_q max_v U(theta_i, v, q, f(theta_i)) >= f(theta) on a dense in-tile grid."""
    r = 1 / 16
    for c in [(-1.0, -1.0), (0.0, -0.5), (-2.5, -2.9)]:
        c = np.array(c)
        corners = np.array([[sx * r, sy * r] for sx in (-1, 1) for sy in (-1, 1)])
        a = _exact_tie_binom2(c)
        b, _ = O.tile_bound("binom", c[None], corners[None], np.array([a]))
        g = np.linspace(-r, r, 7)
        worst = max(_exact_tie_binom2(c + np.array([dx, dy])) for dx in g for dy in g)
        assert b[0] >= worst


def test_theorem1_ztest_tiles_slack_nonnegative():
    th = -1 + (2 * np.arange(64) + 1) / 128
    r = 1 / 128
    b, _ = O.tile_bound("normal", th[:, None], np.tile(np.array([[[r], [-r]]]), (64, 1, 1)), f_z(th))
    g = np.linspace(-r, r, 21)
    worst = np.max(f_z(th[:, None] + g[None, :]), axis=1)
    assert np.all(b - worst >= 0.0)


def test_vertices_dominate_interior_theorem3():
    rng = np.random.default_rng(1)
    c = np.array([-0.7, -1.1])
    corners = np.array([[sx, sy] for sx in (-0.2, 0.2) for sy in (-0.2, 0.2)])
    for q in (1.3, 5.0, 60.0):
        vmax = max(O.log_tilt("binom", c, v, q, 0.02) for v in corners)
        for _ in range(300):
            v = rng.uniform(-0.2, 0.2, 2)
            assert O.log_tilt("binom", c, v, q, 0.02) <= vmax + 1e-12


def test_inverse_round_trip():
    """alpha' from the inverse bound, pushed through the forward bound at its q*, gives alpha."""
    th = np.array([[0.2, -0.4]])
    V = np.array([[[sx * 0.05, sy * 0.05] for sx in (-1, 1) for sy in (-1, 1)]])
    ap, q = O.tile_inverse("binom", th, V, 0.025)
    back = max(math.exp(O.log_tilt("binom", th[0], v, q[0], ap[0])) for v in V[0])
    assert back == pytest.approx(0.025, rel=1e-9)


def test_clopper_pearson_closed_forms():
    N, d = 10_000, 0.01
    assert O.cp_upper(np.array([0]), np.array([N]), d)[0] == pytest.approx(1 - d ** (1 / N), rel=1e-12)
    assert O.cp_upper(np.array([N - 1]), np.array([N]), d)[0] == pytest.approx((1 - d) ** (1 / N), rel=1e-12)
    assert O.cp_upper(np.array([N]), np.array([N]), d)[0] == 1.0


@pytest.mark.parametrize("N,R", [(200, 0), (200, 3), (200, 100), (2000, 49), (10_000, 250)])
def test_clopper_pearson_tail_identity_mpmath(N, R):
    mp.mp.dps = 50
    d = 0.01
    u = mp.mpf(float(O.cp_upper(np.array([R]), np.array([N]), d)[0]))
    tail = mp.fsum(mp.binomial(N, j) * u**j * (1 - u) ** (N - j) for j in range(R + 1))
    assert float(tail) == pytest.approx(d, rel=1e-9)


def test_subtiles_binom2_diagonal_triangle():
    subs = O.subtiles("binom2", np.array([[0.5, 0.5], [0.5, 0.25], [0.25, 0.5]]), np.full((3, 2), 0.125))
    assert [s[0] for s in subs] == [0, 1]            # the box above the diagonal meets no null
    tri = subs[0][2]
    assert len(tri) == 3
    expect = {(0.375, 0.375), (0.625, 0.375), (0.625, 0.625)}
    assert {tuple(np.round(v, 12)) for v in tri} == expect
    assert len(subs[1][2]) == 4


def test_subtiles_hier4_partition_by_sampling():
    """Each box is split into pieces box ∩ P(b); a dense sample of the box must land, for
    every b that owns sampled points, in a sub-tile with that b, and every sub-tile must own points."""
    rng = np.random.default_rng(2)
    cs = -1 + (2 * np.arange(4) + 1) / 4
    boxes = np.array(list(itertools.product(cs, repeat=4)))
    r = 0.25
    subs = O.subtiles("hier4", boxes, np.full_like(boxes, r))
    by_box = {}
    for i, b, V, _ in subs:
        by_box.setdefault(i, set()).add(b)
    for i, c in enumerate(boxes):
        x = c + rng.uniform(-r, r, (4000, 4))
        b = ((x[:, 1] <= x[:, 0]) * 1 + (x[:, 2] <= x[:, 0]) * 2 + (x[:, 3] <= x[:, 0]) * 4)
        seen = set(np.unique(b[b > 0]).tolist())
        assert seen == by_box.get(i, set())


# ------------------------------------------------------------- lower bounds (Remark 2)
def test_cp_lower_scipy_and_symmetry():
    from scipy import special
    N = np.array([10, 100, 10000, 10000, 37])
    R = np.array([3, 0, 250, 10000, 37])
    lo = O.cp_lower(R, N, 0.01)
    assert lo[1] == 0.0
    ok = R > 0
    np.testing.assert_allclose(lo[ok], special.betaincinv(R[ok], N[ok] - R[ok] + 1, 0.01), rtol=1e-12)
    # lower bound of p from R successes = 1 - upper bound of 1 - p from N - R successes
    np.testing.assert_allclose(lo, 1.0 - O.cp_upper(N - R, N, 0.01), rtol=0, atol=1e-12)
    # R = N: Beta(N, 1) quantile = delta^(1/N)
    assert lo[3] == pytest.approx(0.01 ** (1 / 10000), rel=1e-12)


@pytest.mark.parametrize("r", [1 / 128, 0.05, 0.25])
def test_lower_tilt_bound_under_exact_power(r):
    """With the exact f(theta0), the tilewise lower bound is below the exact z-test power at
    every point of the tile (zero exceptions)."""
    from scipy import stats
    th0 = np.linspace(-1.0, 0.5, 31)[:, None]
    V = np.stack([np.full((31, 1), -r), np.full((31, 1), r)], axis=1)
    f0 = stats.norm.cdf(th0[:, 0] - 1.96)
    lb, _ = O.tile_lower("normal", th0, V, f0)
    assert np.all(lb <= f0 + 1e-15)
    for i in range(31):
        x = np.linspace(th0[i, 0] - r, th0[i, 0] + r, 401)
        assert np.all(stats.norm.cdf(x - 1.96) >= lb[i] - 1e-15)


def test_lower_tilt_bound_two_arm_exact():
    """2-arm pooled z design, exact TIE by enumeration: lower bound below the exact TIE at
    vertices and interior points of boxes and diagonal triangles."""
    from test_oracle_taylor import _binom2_exact
    theta = np.array([[-0.5, -0.5], [0.3, -0.2], [-1.2, -1.6]])
    radii = np.full((3, 2), 0.1)
    subs = O.subtiles("binom2", theta, radii)
    box = np.array([s[0] for s in subs])
    f0 = np.array([_binom2_exact(t)[0] for t in theta[box]])
    lb, _ = O.tile_lower("binom", theta[box], O._pad_vertices(subs, theta), f0)
    rng = np.random.default_rng(1)
    for t, (i, b, verts, _) in enumerate(subs):
        pts = list(verts) + [rng.dirichlet(np.ones(len(verts))) @ verts for _ in range(20)]
        for x in pts:
            assert _binom2_exact(x)[0] >= lb[t] - 1e-12
        assert lb[t] <= f0[t]
