"""Pins of the oracle's adaptive gridding (pilot runs choose tile sizes and simulation counts,
Section 10.2), against geometry and the z-test's closed forms rather than the rule itself:

- a split partitions its box (sampled points fall in exactly one child, volumes add up);
- adaptive validation of the z-test: the final boxes tile the domain exactly, every box meets
  the target or is stuck at the limits, the final bounds cover the exact power
  1 - Phi(1.96 - theta) at each box's worst point, and far fewer simulations are spent than a
  uniform grid at the finest size and the largest N would take;
- adaptive calibration of the z-test: the calibrated threshold moves towards the exact level
  alpha test, -lambda* in [z_{1-alpha}, z_{1-alpha} + 0.06], and never away from it;
- the two decision rules on cases whose answer the definitions fix (a wide tile with many
  simulations splits; a narrow tile with few simulations doubles N; limits give "stuck").
"""
import numpy as np
import pytest
from scipy import stats

import oracle as O
from oracle import adagrid as A


@pytest.mark.parametrize("d", [1, 2, 4])
def test_split_partitions_the_box(d):
    rng = np.random.default_rng(d)
    th = rng.uniform(-1, 1, d)
    r = rng.uniform(0.01, 0.3, d)
    kids = A.split_box(th, r)
    assert len(kids) == 2 ** d
    assert np.prod(2 * r) == pytest.approx(sum(np.prod(2 * kr) for _, kr in kids))
    x = th + rng.uniform(-1, 1, (5000, d)) * r
    inside = np.array([[np.all(np.abs(p - kt) <= kr) for kt, kr in kids] for p in x])
    assert np.all(inside.sum(axis=1) == 1)
    for kt, kr in kids:
        assert np.all(kt - kr >= th - r - 1e-15) and np.all(kt + kr <= th + r + 1e-15)


def test_decision_rules_on_clear_cases():
    # validation: box 0 wide with huge N (geometry dominates) -> split; box 1 narrow with few
    # simulations (Monte Carlo dominates) -> double; box 2 already below target -> done;
    # box 3 at both limits -> stuck
    radii = np.array([[0.5], [0.001], [0.1], [0.001]])
    sims = np.array([10 ** 6, 100, 1000, 1024], np.int32)
    bound = np.array([0.20, 0.08, 0.01, 0.2])
    cp = np.array([0.03, 0.075, 0.009, 0.15])
    fhat = np.array([0.029, 0.03, 0.008, 0.149])
    dec = A.decide_validation(radii, sims, np.arange(4), bound, cp, fhat, target=0.05, r_min=0.001, n_max=1024)
    assert list(dec) == [A.SPLIT, A.DOUBLE, A.DONE, A.STUCK]
    # calibration: only the box holding lambda* (margin 0) is critical
    lam = np.array([-2.0, -1.9, -1.5])
    ap = np.array([0.010, 0.024, 0.024])
    N = np.array([10 ** 6, 100, 100])
    dec = A.decide_calibration(np.array([[0.2], [0.2], [0.2]]), N.astype(np.int32), np.arange(3), lam, ap, N,
                               alpha=0.025, margin=0.0, r_min=0.001, n_max=1 << 20)
    assert list(dec) == [A.SPLIT, A.DONE, A.DONE]
    dec = A.decide_calibration(np.array([[0.2], [0.2], [0.2]]), N.astype(np.int32), np.arange(3), lam, ap, N,
                               alpha=0.025, margin=0.15, r_min=0.001, n_max=1 << 20)
    assert list(dec) == [A.SPLIT, A.DOUBLE, A.DONE]      # box 1: slack 0.001 < spread 0.015


def test_ztest_adaptive_validation():
    th = np.array([[-0.875], [-0.625], [-0.375], [-0.125]])
    rd = np.full((4, 1), 0.125)
    sims = np.full(4, 500, np.int32)
    r_min, n_max, target = 1.0 / 512, 1 << 16, 0.03
    out = A.run("ztest1", th, rd, sims, seed=3, mode="validate", target=target, delta=0.01, r_min=r_min,
                n_max=n_max, max_rounds=20)
    T, R, S, dec = out["theta"][:, 0], out["radii"][:, 0], out["sims"], out["decision"]
    order = np.argsort(T)
    lo, hi = (T - R)[order], (T + R)[order]
    assert lo[0] == pytest.approx(-1.0) and hi[-1] == pytest.approx(0.0)
    np.testing.assert_allclose(lo[1:], hi[:-1], rtol=0, atol=1e-15)       # contiguous, no overlap
    U = np.zeros(len(T))
    for t, b in enumerate(out["box_of_tile"]):
        U[b] = max(U[b], out["tiles"]["bound"][t])
    assert np.all((U <= target) | (dec == A.STUCK))
    assert np.all(dec != A.SPLIT) and np.all(dec != A.DOUBLE)
    exact = stats.norm.sf(1.96 - (T + R))                                   # worst point of each box
    assert np.sum(exact > U + 1e-15) <= 1                                   # valid w.p. 1 - delta each
    spent = sum(h[4] for h in out["history"])
    uniform = (1.0 / (2 * r_min)) * n_max
    print(f"boxes {len(T)}, rounds {out['rounds']}, simulations {spent}, uniform {uniform:.3g}")
    assert spent * 10 < uniform


def test_ztest_adaptive_calibration():
    th = (np.arange(8) * 0.125 - 1.0 + 0.0625)[:, None]
    rd = np.full((8, 1), 0.0625)
    sims = np.full(8, 1000, np.int32)
    alpha = 0.025
    first = O.calibrate("ztest1", th, rd, sims, 5, alpha)
    out = A.run("ztest1", th, rd, sims, seed=5, mode="calibrate", alpha=alpha, margin=0.0, r_min=1.0 / 1024,
                n_max=1 << 17, max_rounds=40)
    lam = out["tiles"]["lam"]
    z = stats.norm.ppf(1 - alpha)
    print(f"-lambda*: first grid {-first['lam_global']:.4f}, adaptive {-lam.min():.4f} after "
          f"{out['rounds']} rounds, {len(out['sims'])} boxes")
    assert z <= -lam.min() <= z + 0.06
    assert -lam.min() <= -first["lam_global"] + 1e-12
    # the exact Type I Error of the calibrated test at the worst null point theta = 0
    assert stats.norm.sf(-lam.min()) <= alpha
