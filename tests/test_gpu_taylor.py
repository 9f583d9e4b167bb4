"""GPU: Taylor comparison bound and gradient-guided worst-case vertex (Section 4.3) through the
C ABI vs the oracle, from exact values (2-arm enumeration) and from the library's own
estimates (Clopper-Pearson bound and score gradient of one validation pass), and the search's
purpose: the chosen vertex carries (nearly) the largest exact Type I Error of the tile.

Vertex orders of the two enumerations may differ, so chosen vertices are compared as points.
"""
import numpy as np
import pytest
import torch

import oracle as O
import paper_2212_10042_amd as cse
import workloads as W
from test_oracle_taylor import _binom2_exact

pytestmark = pytest.mark.gpu


def _np(t):
    return t.detach().cpu().numpy()


def _dev(a):
    return torch.tensor(np.ascontiguousarray(a, np.float64), device="cuda")


def _oracle(design, w, subs, f, g):
    box = np.array([s[0] for s in subs])
    th = w["theta"][box]
    V = O._pad_vertices(subs, w["theta"])
    ub, j = O.taylor_bound(O.family_of(design), th, w["radii"][box], V, f, g, n=O.n_of(design))
    pts = th + V[np.arange(len(j)), j]
    return ub, pts


def _check_points(design, w, subs, f, g, got):
    """The chosen vertex must attain the tile's maximum of the Taylor model (the two
    enumerations may order vertices differently, so exact ties may pick different ones)."""
    box = np.array([s[0] for s in subs])
    th = w["theta"][box]
    h = O.curvature_bound(O.family_of(design), th, w["radii"][box], n=O.n_of(design))
    ub, pts = _oracle(design, w, subs, f, g)
    for t, s in enumerate(subs):
        v = got[t] - th[t]
        assert np.min(np.max(np.abs(s[2] - got[t]), axis=1)) < 1e-12   # it is a vertex of the tile
        val = f[t] + v @ g[t] + 0.5 * (v * v) @ h[t]
        if ub[t] < 1.0:   # below the clip the model's value at the chosen vertex is the bound
            assert val == pytest.approx(ub[t], rel=1e-12, abs=1e-15)


def test_binom2_exact_values_and_worst_vertex():
    w = W.binom2_grid(10, 100, lo=-1.5, hi=0.5, seed=0)
    P = cse.Platten.create("binom2", w["theta"], w["radii"], w["sims"])
    subs = O.subtiles("binom2", w["theta"], w["radii"])
    box = np.array([s[0] for s in subs])
    fg = [_binom2_exact(t) for t in w["theta"][box]]
    f = np.array([a for a, _ in fg])
    g = np.array([b for _, b in fg])
    print(f"[taylor] binom2 exact values, {len(subs)} tiles", flush=True)
    o = P.taylor(_dev(f), _dev(g))
    torch.cuda.synchronize()
    ub, pts = _oracle("binom2", w, subs, f, g)
    np.testing.assert_allclose(_np(o["bound"]), ub, rtol=1e-13, atol=0)
    _check_points("binom2", w, subs, f, g, _np(o["point"]))
    # the bound covers the exact TIE at every vertex of every tile
    for t, s in enumerate(subs):
        assert max(_binom2_exact(v)[0] for v in s[2]) <= _np(o["bound"])[t] + 1e-12
    P.close()


def test_binom2_estimates_and_search():
    """From one validation pass: the Taylor bound on (cp_upper, score gradient) equals the
    oracle's on the same (exact integer) counts, and the vertex the estimated gradient points to
    carries the tile's largest exact TIE up to a small tolerance on most tiles."""
    w = W.binom2_grid(12, 20000, lo=-1.0, hi=0.5, seed=2)
    P = cse.Platten.create("binom2", w["theta"], w["radii"], w["sims"])
    v = P.validate(seed=2, delta=0.01)
    o = P.taylor(v["cp_upper"], v["grad"])
    torch.cuda.synchronize()
    subs = O.subtiles("binom2", w["theta"], w["radii"])
    ov = O.validate("binom2", w["theta"], w["radii"], w["sims"], 2, 0.01)
    assert np.array_equal(_np(v["reject"]), ov["R"])
    gO = O.score_gradient("binom2", w["theta"][ov["box"]], ov["R"], ov["score"], ov["N"])
    ub, pts = _oracle("binom2", w, subs, ov["cp"], gO)
    np.testing.assert_allclose(_np(o["bound"]), ub, rtol=1e-12, atol=0)
    _check_points("binom2", w, subs, ov["cp"], gO, _np(o["point"]))
    good = []
    for t, s in enumerate(subs):
        exact = np.array([_binom2_exact(vx)[0] for vx in s[2]])
        chosen = _binom2_exact(_np(o["point"])[t])[0]
        good.append(chosen >= exact.max() - 2e-4)
    print(f"[taylor] worst vertex found on {np.mean(good):.3f} of {len(subs)} tiles", flush=True)
    assert np.mean(good) >= 0.9
    P.close()


@pytest.mark.parametrize("design", ["ztest1", "hier4", "phase23"])
def test_other_designs_vs_oracle(design):
    rng = np.random.default_rng(4)
    if design == "ztest1":
        w = W.ztest_1d(30, 100)
    elif design == "hier4":
        w = W.hier4_grid(2, 100, seed=1)
    else:
        w = W.phase23_grid((2, 2, 1, 1), 100, seed=1)
    P = cse.Platten.create(design, w["theta"], w["radii"], w["sims"], cut=w.get("cut"))
    subs = O.subtiles(design, w["theta"], w["radii"])
    d = w["theta"].shape[1]
    f = rng.uniform(0.0, 0.05, len(subs))
    g = rng.normal(0.0, 0.1, (len(subs), d))
    print(f"[taylor] {design}: {len(subs)} tiles", flush=True)
    o = P.taylor(_dev(f), _dev(g))
    torch.cuda.synchronize()
    ub, pts = _oracle(design, w, subs, f, g)
    np.testing.assert_allclose(_np(o["bound"]), ub, rtol=1e-13, atol=0)
    _check_points(design, w, subs, f, g, _np(o["point"]))
    P.close()
