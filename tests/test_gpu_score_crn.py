"""GPU: the score-function gradient of the 4-arm and basket designs (Example 1: the sum over
rejecting simulations of the arm counts, minus R n expit(theta), over N) against the rejection
counts themselves under common random numbers.

Every simulation uses the same Philox words at every point, so along arm a the count
difference R(theta + h e_a) - R(theta - h e_a) is N times the integral of the rejection rate's
derivative over [theta - h, theta + h] plus the noise of the simulations whose decision
differs between the two ends.  The score estimates at theta - h, theta and theta + h (one pass)
give that integral by Simpson's rule.  Tolerance: 4.5 times a bound on both standard errors --
sqrt(R(+) + R(-)) for the count difference (at most every rejection flips) and
35 sqrt(R) / N for each score estimate (each term of the sum is at most 35 in magnitude).
Boxes are tiny (half-width 1e-4) and keep one configuration b over the whole segment.
"""
import math

import numpy as np
import pytest
import torch

import paper_2212_10042_amd as cse

pytestmark = pytest.mark.gpu

H = 0.05
N = 1 << 18


def _np(t):
    return t.detach().cpu().numpy()


def _segments(pts):
    """Boxes at each point and at point +- H e_a for every arm a."""
    rows = [pts]
    for a in range(4):
        for sg in (1.0, -1.0):
            q = pts.copy()
            q[:, a] += sg * H
            rows.append(q)
    return np.concatenate(rows)


def _check(kind, pts, seed, theta0=None):
    m = pts.shape[0]
    th = _segments(pts)
    P = cse.Platten.create(kind, th, np.full_like(th, 1e-4), np.full(th.shape[0], N, np.int32), theta0=theta0)
    box = P.tiles["box"]
    assert np.array_equal(box, np.arange(th.shape[0])), "one tile per box (no box straddles a boundary)"
    cfg = P.tiles["cfg"]
    o = P.simulate(seed)
    torch.cuda.synchronize()
    R = _np(o["reject"]).astype(np.float64)
    g = _np(o["grad"])
    print(f"[score-crn] {kind}: {m} points, rejection rates {np.round(R[:m] / N, 4).tolist()}", flush=True)
    assert np.all(R[:m] > 100), "each point must reject often enough to test"
    checked = 0
    for a in range(4):
        ip = slice(m * (1 + 2 * a), m * (2 + 2 * a))
        im = slice(m * (2 + 2 * a), m * (3 + 2 * a))
        assert np.array_equal(cfg[ip], cfg[:m]) and np.array_equal(cfg[im], cfg[:m])
        diff = R[ip] - R[im]
        simpson = N * 2 * H * (g[im, a] + 4 * g[:m, a] + g[ip, a]) / 6.0
        se = np.sqrt(R[ip] + R[im]) + 2 * H / 6.0 * 35 * (np.sqrt(R[im]) + 4 * np.sqrt(R[:m]) + np.sqrt(R[ip]))
        z = (diff - simpson) / se
        print(f"[score-crn] {kind} arm {a}: diff {diff.tolist()}, Simpson {np.round(simpson, 1).tolist()}, "
              f"|z| max {np.abs(z).max():.2f}", flush=True)
        assert np.all(np.abs(z) < 4.5)
        checked += int(np.sum(np.abs(diff) > 3 * np.sqrt(R[ip] + R[im])))
    # the check has teeth: several segments move the rejection count well beyond its noise
    assert checked >= 3
    P.close()


def test_hier4_score_gradient_vs_crn_differences():
    # control arm 0 against treatments 1..3; points in the null of one, two and three arms,
    # every treatment at least 0.2 from the control so the segment keeps its configuration
    pts = np.array([[0.3, 0.0, -0.4, 0.8],
                    [0.2, -0.1, -0.3, -0.5],
                    [-0.2, 0.3, -0.6, 0.1]])
    _check("hier4", pts, seed=21)


def test_basket_score_gradient_vs_crn_differences():
    # every arm against p0 = 15% (logit -1.7346): arms in the null where theta_a <= -1.7346
    t0 = math.log(0.15 / 0.85)
    pts = np.array([[t0 - 0.3, t0 + 0.8, t0 + 0.6, t0 + 1.0],
                    [t0 - 0.4, t0 - 0.3, t0 + 0.9, t0 + 0.7],
                    [t0 - 0.5, t0 + 1.2, t0 - 0.25, t0 + 0.5]])
    _check("basket4", pts, seed=22)
