"""Pins of the oracle's Taylor comparison bound and worst-vertex choice (Section 4.3), each
against something other than the bound's own formula:

- the z-test with the exact f = Phi(theta - 1.96) and f': the bound covers the exact power
  function on a dense grid of every tile;
- the paper's comparison (Section 4.3): at theta0 = -0.25 and distance 0.25 the Taylor bound is
  far looser than the printed optimised Tilt-Bound 2.73%, while for very small distances it is
  the tighter one;
- 2-arm pooled z design: exact TIE and gradient by enumeration of the 36 x 36 outcomes; the
  bound covers the exact TIE at the vertices and a dense set of points of boxes and diagonal
  triangles;
- the curvature bound against a brute-force maximum of n p (1 - p) over the box.
"""

import numpy as np
import pytest
from scipy import stats

import oracle as O
from conftest import read_golden

N35 = 35


def _ztest_f(th):
    return stats.norm.cdf(th - 1.96)


def test_curvature_bound_brute_force():
    rng = np.random.default_rng(2)
    th = rng.uniform(-3, 3, (40, 2))
    r = rng.uniform(0.01, 0.8, (40, 2))
    h = O.curvature_bound("binom", th, r)
    for i in range(40):
        for a in range(2):
            x = np.linspace(th[i, a] - r[i, a], th[i, a] + r[i, a], 20001)
            p = 1 / (1 + np.exp(-x))
            assert h[i, a] == pytest.approx(np.max(N35 * p * (1 - p)), rel=1e-6)
    assert np.all(O.curvature_bound("normal", th[:, :1], r[:, :1]) == 1.0)


@pytest.mark.parametrize("r", [1 / 128, 0.05, 0.25])
def test_ztest_taylor_covers_exact_power(r):
    th0 = np.linspace(-1.0, 0.3, 27)[:, None]
    V = np.array([[[-r]], [[r]]]).transpose(1, 0, 2).repeat(len(th0), axis=0)   # [m, 2, 1]
    f = _ztest_f(th0[:, 0])
    g = stats.norm.pdf(th0 - 1.96)
    ub, j = O.taylor_bound("normal", th0, np.full_like(th0, r), V, f, g)
    for i in range(len(th0)):
        x = np.linspace(th0[i, 0] - r, th0[i, 0] + r, 401)
        assert np.all(_ztest_f(x) <= ub[i] + 1e-15)
    # f is increasing: the worst vertex is the upper end of every tile
    assert np.all(j == 1)


def test_paper_comparison_with_tilt_bound():
    rows = read_golden("paper_tilt_values.txt")
    tilt = float(rows[0][3]) / 100.0   # optimised Tilt-Bound at theta0 = -0.25, v = 0.25 (2.73%)
    th0, v = -0.25, 0.25
    f, g = _ztest_f(th0), stats.norm.pdf(th0 - 1.96)
    ub, _ = O.taylor_bound("normal", np.array([[th0]]), np.array([[v]]), np.array([[[v]]]), [f], [[g]])
    assert ub[0] > tilt > _ztest_f(th0 + v)
    # for a very small distance the Taylor bound is the tighter one
    vs = 0.002
    ubs, _ = O.taylor_bound("normal", np.array([[th0]]), np.array([[vs]]), np.array([[[vs]]]), [f], [[g]])
    tilts, _ = O.tile_bound("normal", np.array([[th0]]), np.array([[[vs]]]), np.array([f]))
    assert _ztest_f(th0 + vs) <= ubs[0] < tilts[0]


def _binom2_exact(th):
    """Exact TIE and gradient of the pooled-z 2-arm design at theta = (theta0, theta1)."""
    y = np.arange(N35 + 1)
    z = np.array([[O.pooled_z(a, b) for b in y] for a in y])
    rej = z > 1.96
    p = 1 / (1 + np.exp(-np.asarray(th)))
    P0 = stats.binom.pmf(y, N35, p[0])
    P1 = stats.binom.pmf(y, N35, p[1])
    joint = P0[:, None] * P1[None, :] * rej
    f = joint.sum()
    g0 = (joint * (y[:, None] - N35 * p[0])).sum()
    g1 = (joint * (y[None, :] - N35 * p[1])).sum()
    return f, np.array([g0, g1])


def test_binom2_taylor_covers_exact_tie():
    w = {"theta": np.array([[-0.5, -0.5], [0.3, -0.2], [-1.2, -1.6], [0.0, 0.0]]),
         "radii": np.full((4, 2), 0.12)}
    subs = O.subtiles("binom2", w["theta"], w["radii"])
    box = np.array([s[0] for s in subs])
    th = w["theta"][box]
    fg = [_binom2_exact(t) for t in th]
    f = np.array([a for a, _ in fg])
    g = np.array([b for _, b in fg])
    V = O._pad_vertices(subs, w["theta"])
    ub, j = O.taylor_bound("binom", th, w["radii"][box], V, f, g)
    rng = np.random.default_rng(0)
    for t, (i, b, verts, _) in enumerate(subs):
        pts = list(verts)
        # dense points of the tile: convex combinations of its vertices
        for _ in range(30):
            lam = rng.dirichlet(np.ones(len(verts)))
            pts.append(lam @ verts)
        for x in pts:
            assert _binom2_exact(x)[0] <= ub[t] + 1e-12
        # the chosen vertex maximises the quadratic model over the vertices
        model = f[t] + (verts - th[t]) @ g[t] + 0.5 * ((verts - th[t]) ** 2) @ O.curvature_bound(
            "binom", th[t:t + 1], w["radii"][box][t:t + 1])[0]
        assert j[t] == int(np.argmax(model))
    assert any(len(s[2]) == 3 for s in subs)   # a diagonal triangle is among the tiles
