"""Pins of the oracle's Phase II/III selection design (Section 10.2 and the design appendix;
reading in oracle_phase23.c), each against something other than the oracle's own formula:

- the 16-point Gauss-Hermite rule against numpy's hermgauss, z95 against scipy's norm.ppf;
- the posterior summary with equal sample sizes reduces to the 4-arm posterior pinned in
  test_oracle_hier.py; with unequal sizes its node modes maximise the scipy.stats log-density,
  and at large n its mixture mean / variance match quadrature of the exact posterior;
- p_best against scipy.integrate.quad of its defining integral, summing to one, 1/4 under
  symmetry; p_success against a Monte Carlo of the Gaussian predictive it describes and its
  infinite-data limit P(d > 0);
- every simulated trial replayed in Python against the protocol: allocations, the words its
  responses come from (Philox, pinned by its known-answer test), each look's decision from the
  separately pinned summary / p_best / p_success, the calibration statistic, and the caps of
  350 patients per arm and 800 in total;
- the score-function gradient with observed counts and sizes, (sum_rej y_a - sum_rej n_a expit
  theta_a) / N, against the change of the rejection rate itself: under common random numbers
  the count difference R(theta + h e_a) - R(theta - h e_a) must equal Simpson's integral of the
  score estimate over [theta - h, theta + h] within the paired per-trial standard error, on every
  arm (a wrong sample size such as the embedded 350, a sign or a dropped arm fails by > 10 or
  > 3 standard errors).
"""
import itertools
import math
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest
from scipy import integrate, optimize, special, stats

import oracle as O

D = 4


def test_gauss_hermite_rule_matches_numpy():
    x, w = O.gh16()
    xr, wr = np.polynomial.hermite.hermgauss(16)
    np.testing.assert_allclose(x, xr, rtol=0, atol=1e-13)
    np.testing.assert_allclose(w, wr, rtol=1e-12, atol=0)


def test_z95():
    assert O.z95() == pytest.approx(stats.norm.ppf(0.95), abs=1e-14)


@pytest.mark.parametrize("y", [(10, 14, 3, 30), (0, 35, 17, 2)])
def test_summary_equal_sizes_reduces_to_pinned_posterior(y):
    s = O.hier4_summary(y, [35] * 4)
    np.testing.assert_allclose(s["P"], O.hier4_posterior(y), rtol=0, atol=1e-15)
    np.testing.assert_allclose(s["Sc"], 1.0 - s["P"], rtol=0, atol=1e-14)
    np.testing.assert_allclose(s["dmean"], s["mean"][1:] - s["mean"][0], rtol=0, atol=1e-14)
    assert np.all(s["var"] > 0) and np.all(s["dvar"] > 0)


def _logdens(th, y, n, s2):
    cov = s2 * np.eye(4) + 100.0 * np.ones((4, 4))
    p = 1.0 / (1.0 + np.exp(-th))
    return (np.sum(stats.binom.logpmf(y, n, p))
            + stats.multivariate_normal(mean=np.full(4, -1.34), cov=cov).logpdf(th))


def test_unequal_sizes_node_modes_maximise_density():
    y = np.array([20, 61, 40, 9])
    n = np.array([150, 150, 83, 50])
    mode = np.zeros((90, 4))
    lw = np.zeros(90)
    out = np.zeros(20)
    O.lib().orc_hier4_summary(O._p(y.astype(np.int32)), O._p(n.astype(np.int32)), O._p(out), O._p(mode), O._p(lw))
    for j in (0, 40, 89):
        ls2 = -13.815510557964274 + j * (6.907755278982137 + 13.815510557964274) / 89
        f = lambda th: _logdens(th, y, n, math.exp(ls2))
        res = optimize.minimize(lambda th: -f(th), mode[j] + 0.2, method="BFGS", options=dict(gtol=1e-10))
        assert f(mode[j]) >= -res.fun - 1e-9
        h = 1e-4
        for a in range(4):
            e = np.zeros(4)
            e[a] = h
            g = (f(mode[j] + e) - f(mode[j] - e)) / (2 * h)
            c = (f(mode[j] + e) - 2 * f(mode[j]) + f(mode[j] - e)) / (h * h)
            assert c < 0 and abs(g / c) < 1e-5


def test_mixture_moments_match_quadrature_at_large_n():
    """At n ~ 1e3 per arm the Laplace mixture's mean and variance of each theta_a and of
    theta_i - theta_0 must match adaptive Gauss-Hermite quadrature of the exact posterior
    (node weights from the quadrature evidence) to O(1/n)."""
    y = np.array([700, 1190, 300, 520])
    n = np.array([1500, 2000, 800, 1200])
    s = O.hier4_summary(y, n)
    z, w = np.polynomial.hermite.hermgauss(10)
    Z = np.array(list(itertools.product(z, repeat=4)))
    W = np.prod(np.array(list(itertools.product(w, repeat=4))), axis=1)
    logs2 = np.linspace(-13.815510557964274, 6.907755278982137, 90)
    h = logs2[1] - logs2[0]
    evid, m1, m2, d1, d2 = [], [], [], [], []
    for j, ls2 in enumerate(logs2):
        s2 = math.exp(ls2)
        cov = s2 * np.eye(4) + 100.0 * np.ones((4, 4))
        Q = np.linalg.inv(cov)
        th = np.log((y + 0.5) / (n - y + 0.5))
        for _ in range(100):
            p = special.expit(th)
            g = y - n * p - Q @ (th + 1.34)
            H = -np.diag(n * p * (1 - p)) - Q
            st = np.linalg.solve(H, g)
            th = th - st
            if np.abs(st).max() < 1e-12:
                break
        p = special.expit(th)
        C = np.linalg.inv(np.diag(n * p * (1 - p)) + Q)
        L = np.linalg.cholesky(C)
        X = th + math.sqrt(2.0) * Z @ L.T
        ll = (stats.binom.logpmf(y[None, :], n, special.expit(X)).sum(axis=1)
              + stats.multivariate_normal(mean=np.full(4, -1.34), cov=cov).logpdf(X))
        lf = ll + np.sum(Z * Z, axis=1)
        mx = lf.max()
        wt = W * np.exp(lf - mx)
        tot = wt.sum()
        logprior = 0.0005 * math.log(0.000005) - math.lgamma(0.0005) - 1.0005 * ls2 - 0.000005 / s2
        trap = (0.5 if j in (0, 89) else 1.0) * h
        evid.append(mx + math.log(tot) + math.log(abs(np.linalg.det(math.sqrt(2.0) * L))) + logprior
                    + math.log(trap) + ls2)
        m1.append((wt[:, None] * X).sum(0) / tot)
        m2.append((wt[:, None] * X * X).sum(0) / tot)
        dd = X[:, 1:] - X[:, :1]
        d1.append((wt[:, None] * dd).sum(0) / tot)
        d2.append((wt[:, None] * dd * dd).sum(0) / tot)
    evid = np.array(evid)
    pi = np.exp(evid - evid.max())
    pi /= pi.sum()
    mean = pi @ np.array(m1)
    var = pi @ np.array(m2) - mean ** 2
    dmean = pi @ np.array(d1)
    dvar = pi @ np.array(d2) - dmean ** 2
    np.testing.assert_allclose(s["mean"], mean, atol=3e-3)
    np.testing.assert_allclose(s["var"], var, rtol=0.05)
    np.testing.assert_allclose(s["dmean"], dmean, atol=3e-3)
    np.testing.assert_allclose(s["dvar"], dvar, rtol=0.05)


@pytest.mark.parametrize("m,v", [([0.1, 0.3, -0.2, 0.25], [0.04, 0.02, 0.05, 0.03]),
                                 ([-0.5, -0.45, -0.7, -0.2], [0.01, 0.015, 0.02, 0.012])])
def test_pbest_matches_integral(m, v):
    """The 16-point rule built from numpy's nodes gives the same numbers to rounding; the
    integral itself (scipy quad) is matched within the rule's error on these integrands."""
    pb = O.pbest(m, v)
    m = np.array(m)
    s = np.sqrt(v)
    xr, wr = np.polynomial.hermite.hermgauss(16)
    for i in range(4):
        f = lambda t: stats.norm.pdf(t, m[i], s[i]) * np.prod(
            [stats.norm.cdf((t - m[k]) / s[k]) for k in range(4) if k != i], axis=0)
        ref, _ = integrate.quad(f, m[i] - 12 * s[i], m[i] + 12 * s[i], epsabs=1e-13, epsrel=1e-12, limit=200)
        assert pb[i] == pytest.approx(ref, abs=5e-5)
        t = m[i] + math.sqrt(2.0) * s[i] * xr
        rule = np.sum(wr * np.prod([stats.norm.cdf((t - m[k]) / s[k]) for k in range(4) if k != i], axis=0))
        assert pb[i] == pytest.approx(rule / math.sqrt(math.pi), abs=1e-12)
    assert pb.sum() == pytest.approx(1.0, abs=1e-4)


def test_pbest_symmetric_quarter():
    """Equal marginals: all four equal exactly; each is int phi Phi^3 = 1/4 up to the rule's error."""
    pb = O.pbest([0.2] * 4, [0.03] * 4)
    assert np.all(pb == pb[0])
    np.testing.assert_allclose(pb, 0.25, atol=1e-6)


@pytest.mark.parametrize("md,vd,m0,mi,madd", [(0.3, 0.09, -0.2, 0.1, 200), (0.05, 0.04, 0.0, 0.05, 100),
                                              (0.6, 0.05, 0.4, 1.0, 200)])
def test_psucc_matches_predictive_monte_carlo(md, vd, m0, mi, madd):
    rng = np.random.default_rng(5)
    K = 2_000_000
    V = 1.0 / (madd * special.expit(mi) * (1 - special.expit(mi))) + \
        1.0 / (madd * special.expit(m0) * (1 - special.expit(m0)))
    d = rng.normal(md, math.sqrt(vd), K)            # the difference under the current posterior
    dhat = d + rng.normal(0.0, math.sqrt(V), K)     # what the added patients estimate
    prec = 1.0 / vd + 1.0 / V
    mf = (md / vd + dhat / V) / prec
    succ = stats.norm.sf(0.0, mf, math.sqrt(1.0 / prec)) > 0.95
    ref = succ.mean()
    se = math.sqrt(ref * (1 - ref) / K)
    assert abs(O.psucc(md, vd, m0, mi, madd) - ref) < 4 * se + 1e-12


def test_psucc_infinite_data_limit():
    """As the added sample grows, p_success tends to P(d > 0) = Phi(md / sd), with an error
    of order z95 sqrt(V) / sd (the final posterior's own width)."""
    for m_add in (10**5, 10**7, 10**9):
        V = 2.0 / (m_add * 0.25) * (1 + 1e-9)
        err = abs(O.psucc(0.2, 0.04, 0.0, 0.0, m_add) - stats.norm.cdf(0.2 / 0.2))
        assert err < 1.645 * math.sqrt(V) / 0.2 * stats.norm.pdf(1.0) * 1.5


# ----------------------------------------------------------------- the trial, replayed
def _counts(theta, seed, k, n):
    T = [O.bern_threshold(t) for t in theta]
    return [sum(O.word(seed, k, a * 350 + j) < T[a] for j in range(n[a])) for a in range(4)]


def _replay(theta, cfg, seed, k, info, trace, S):
    """Walk the protocol look by look with the pinned building blocks; returns the outcome code
    (0 futility in Phase II, 1 futility at the Phase III interim, 2 early success, 3 final)."""
    outcome, sel, looks = int(info[0]), int(info[1]), int(info[2])
    n_fin, y_fin = list(info[3:7]), list(info[7:11])
    assert max(n_fin) <= 350 and sum(n_fin) <= 800
    assert y_fin == _counts(theta, seed, k, n_fin)
    tr = trace[:looks]
    assert list(tr[0][:4]) == [50] * 4
    for look in range(looks):
        assert list(tr[look][4:]) == _counts(theta, seed, k, tr[look][:4])
    active = [False, True, True, True]
    thr = [0.70, 0.70, 0.60]
    p3 = None
    for look in range(3):
        n, y = tr[look][:4], tr[look][4:]
        s = O.hier4_summary(y, n)
        pb = O.pbest(s["mean"], s["var"])
        ps = {i: O.psucc(s["dmean"][i - 1], s["dvar"][i - 1], s["mean"][0], s["mean"][i], 200)
              for i in range(1, 4) if active[i]}
        q = [i for i in ps if ps[i] > thr[look]]
        if q:
            best = 0   # largest p_best, lowest index on ties; equal data tie exactly
            for i in q:
                if best == 0 or (pb[i] > pb[best] and (y[i], n[i]) != (y[best], n[best])):
                    best = i
            assert sel == best
            p3 = look + 1
            break
        for i in range(1, 4):
            if active[i] and pb[i] < 0.15:
                active[i] = False
        r = sum(active)
        if look == 2 or r == 0:
            assert (sel, outcome, looks) == (0, 0, look + 1) and S == math.inf
            return outcome
        per = 100 // (r + 1)
        assert list(tr[look + 1][:4]) == [n[0] + per] + [n[i] + (per if active[i] else 0) for i in range(1, 4)]
    in_b = (cfg >> (sel - 1)) & 1
    grow = lambda n: [n[0] + 100] + [n[i] + (100 if i == sel else 0) for i in range(1, 4)]
    assert list(tr[p3][:4]) == grow(tr[p3 - 1][:4])
    s3 = O.hier4_summary(tr[p3][4:], tr[p3][:4])
    if s3["P"][sel - 1] > 0.95:
        assert (outcome, looks) == (2, p3 + 1) and S == (-math.inf if in_b else math.inf)
        return outcome
    ps3 = O.psucc(s3["dmean"][sel - 1], s3["dvar"][sel - 1], s3["mean"][0], s3["mean"][sel], 100)
    if ps3 < 0.20:
        assert (outcome, looks) == (1, p3 + 1) and S == math.inf
        return outcome
    assert (outcome, looks) == (3, p3 + 2)
    assert list(tr[p3 + 1][:4]) == grow(tr[p3][:4])
    sf = O.hier4_summary(tr[p3 + 1][4:], tr[p3 + 1][:4])
    assert S == (sf["Sc"][sel - 1] if in_b else math.inf)
    return outcome


def test_trials_follow_the_protocol():
    theta = np.array([[0.0, 0.0, 0.0, 0.0], [-0.3, 0.6, -0.2, 0.1], [0.5, 0.5, 0.45, -0.8],
                      [-0.9, 1.1, 1.0, -0.9]])
    cfg = np.array([7, 4, 3, 0], np.int32)
    sims = np.array([24, 24, 24, 24], np.int32)
    seed = 3
    o = O.sim_phase23(theta, cfg, sims, seed, 0.1, want_S=True, want_info=True, want_trace=True)
    seen = set()
    for t in range(len(theta)):
        for k in range(sims[t]):
            seen.add(_replay(theta[t], int(cfg[t]), seed, k, o["info"][t, k], o["trace"][t, k], o["S"][t, k]))
        rej = o["S"][t, : sims[t]] < 0.1
        assert o["R"][t] == rej.sum()
        np.testing.assert_array_equal(o["sumN"][t], o["info"][t, : sims[t], 3:7][rej].sum(0))
        np.testing.assert_array_equal(o["sumY"][t], o["info"][t, : sims[t], 7:11][rej].sum(0))
    assert {0, 2, 3} <= seen   # futility, early success and final analyses all occur


def test_score_gradient_vs_crn_rate_difference():
    lam, N, h, cfg = 0.06253, 16000, 0.1, 7
    theta = np.array([0.0, 0.1, -0.1, 0.0])
    O.sim_phase23(theta[None], np.array([cfg], np.int32), np.array([1], np.int32), 1, lam)  # rule constants
    pts = [theta] + [theta + s * h * np.eye(D)[a] for a in range(D) for s in (-1, 1)]

    def run(t):   # the C oracle releases the GIL: one thread per point
        return O.sim_phase23(t[None], np.array([cfg], np.int32), np.array([N], np.int32), 5, lam,
                             want_S=True, want_info=True)

    with ThreadPoolExecutor(len(pts)) as ex:
        res = list(ex.map(run, pts))

    def per_trial(o, t, a):
        rej = (o["S"][0] < lam).astype(np.float64)
        n = o["info"][0, :, 3 + a].astype(np.float64)
        y = o["info"][0, :, 7 + a].astype(np.float64)
        return rej, rej * (y - n * special.expit(t[a]))

    for a in range(D):
        rm, sm = per_trial(res[1 + 2 * a], pts[1 + 2 * a], a)
        _, s0 = per_trial(res[0], theta, a)
        rp, sp = per_trial(res[2 + 2 * a], pts[2 + 2 * a], a)
        fd = rp - rm
        Dk = fd - 2 * h * (sm + 4 * s0 + sp) / 6          # paired per trial (same words)
        se = Dk.std() / math.sqrt(N)
        print(f"arm {a}: R difference {fd.mean():+.5f}, integrated score {fd.mean() - Dk.mean():+.5f}, "
              f"z {Dk.mean() / se:+.2f}")
        assert abs(Dk.mean()) < 4.5 * se
        if a < 2:   # the control and the arm that tends to be selected: the change is informative
            assert abs(fd.mean()) > 5 * fd.std() / math.sqrt(N)
