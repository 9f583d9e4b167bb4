"""CPU ORACLE -- test infrastructure only.

A plain, slow, obviously correct FP64 implementation of what the HIP library
computes, written from the paper (Yang, Thompson & Sklar, "Guarantees for
Comprehensive Simulation Assessment of Statistical Methods"):

  * the Monte Carlo loops (Philox stream, draws, statistics, rejection counts,
    score sums) live in plain C (oracle_sim.c, oracle_hier.c), called here
    through ctypes;
  * the bound arithmetic (Clopper-Pearson, Tilt-Bound, its inverse, the
    optimisation over q, the vertex enumeration of clipped tiles, the order
    statistic and the global minimum) is plain numpy/scipy below.

Only tests/, __graft_entry__.smoke() and the CPU-baseline leg of bench.py may
import this package.  It shares no code with paper_2212_10042_amd/ and imports
nothing from it.

Parity status of each function is stated in its docstring ("pinned by" lists
the independent checks in tests/test_oracle_*.py).
"""
from __future__ import annotations

import ctypes
import itertools
import math
import os

import numpy as np
import scipy.special as sps

from . import build as _build

HERE = os.path.dirname(os.path.abspath(__file__))
N_PER_ARM = 35

_lib = None


def lib():
    """Load (building on first use if absent) the oracle's C library."""
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        L = ctypes.CDLL(_build.LIB)
        u32, u64, i32, i64, dbl = (ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int32,
                                   ctypes.c_int64, ctypes.c_double)
        P = ctypes.c_void_p
        L.orc_philox4x32_10.argtypes = [P, P, P]
        L.orc_word.argtypes = [u64, u32, u32]
        L.orc_word.restype = u32
        L.orc_bern_threshold.argtypes = [dbl]
        L.orc_bern_threshold.restype = u32
        L.orc_box_muller.argtypes = [u32, u32]
        L.orc_box_muller.restype = dbl
        L.orc_pooled_z.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int]
        L.orc_pooled_z.restype = dbl
        L.orc_ztest1.argtypes = [i64, P, P, u64, dbl, P, P, P, i64]
        L.orc_binom2.argtypes = [i64, P, P, u64, ctypes.c_int, dbl, P, P, P, i64]
        L.orc_arm_counts.argtypes = [ctypes.c_int, P, i32, u64, ctypes.c_int, P]
        L.orc_hier4_posterior.argtypes = [P, ctypes.c_int, P]
        L.orc_hier4_complement.argtypes = [P, ctypes.c_int, P]
        L.orc_hier4_posterior_full.argtypes = [P, ctypes.c_int, P, P, P, P]
        L.orc_hier4_node.argtypes = [ctypes.c_int, P, P]
        L.orc_hier4_sim.argtypes = [i64, P, P, P, u64, ctypes.c_int, dbl, P, P, P, i64, P]
        L.orc_hier4_table.argtypes = [ctypes.c_int, P, i64, P]
        L.orc_hier4_summary.argtypes = [P, P, P, P, P]
        L.orc_gh16.argtypes = [P, P]
        L.orc_z95.restype = dbl
        L.orc_pbest.argtypes = [P, P, P]
        L.orc_psucc.argtypes = [dbl, dbl, dbl, dbl, ctypes.c_int]
        L.orc_psucc.restype = dbl
        L.orc_tiebreak_u.argtypes = [u64, i64, P]
        L.orc_basket_complement.argtypes = [P, ctypes.c_int, P, P]
        L.orc_basket_table.argtypes = [ctypes.c_int, P, P, i64, P]
        L.orc_basket_sim.argtypes = [i64, P, P, P, u64, ctypes.c_int, P, dbl, P, P, P, i64]
        L.orc_phase23_sim.argtypes = [i64, P, P, P, u64, dbl, P, P, P, P, i64, P, P]
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


# --------------------------------------------------------------- RNG & draws
def philox(ctr, key):
    """Philox4x32-10 block (Salmon et al., SC'11).  Pinned by published known-answer values."""
    c = np.asarray(ctr, np.uint32).copy()
    k = np.asarray(key, np.uint32).copy()
    out = np.zeros(4, np.uint32)
    lib().orc_philox4x32_10(_p(c), _p(k), _p(out))
    return out


def word(seed: int, sim: int, w: int) -> int:
    return int(lib().orc_word(seed, sim, w))


def bern_threshold(theta: float) -> int:
    """round(2^32 expit(theta)) clamped to [0, 2^32-1]: Bernoulli(expit theta) from one word."""
    return int(lib().orc_bern_threshold(float(theta)))


def arm_counts(theta_vec, sims: int, seed: int, n: int = N_PER_ARM) -> np.ndarray:
    """Per-simulation binomial counts Y[k, a] of a d-arm design at one parameter point."""
    th = np.ascontiguousarray(theta_vec, np.float64)
    Y = np.zeros((sims, th.size), np.int32)
    lib().orc_arm_counts(th.size, _p(th), sims, seed, n, _p(Y))
    return Y


def pooled_z(y0: int, y1: int, n: int = N_PER_ARM) -> float:
    return float(lib().orc_pooled_z(y0, y1, n))


# ------------------------------------------------------------------- designs
def sim_ztest1(theta, sims, seed: int, cut: float = 1.96, want_S: bool = False):
    """1-D z-test (Section 4.2, Section 6.4): R, sum of Z over rejections, S = -X."""
    th = np.ascontiguousarray(np.asarray(theta, np.float64).reshape(-1))
    sm = np.ascontiguousarray(sims, np.int32)
    n = th.size
    R = np.zeros(n, np.int32)
    sz = np.zeros(n, np.float64)
    stride = int(sm.max()) if n else 0
    S = np.full((n, stride), np.nan) if want_S else None
    lib().orc_ztest1(n, _p(th), _p(sm), seed, cut, _p(R), _p(sz), _p(S), stride)
    return R, sz, S


def sim_binom2(theta, sims, seed: int, cut: float = 1.96, n: int = N_PER_ARM, want_S: bool = False):
    """2-arm pooled two-proportion z design: R, sumT [n_tiles, 2], S = -z."""
    th = np.ascontiguousarray(np.asarray(theta, np.float64).reshape(-1, 2))
    sm = np.ascontiguousarray(sims, np.int32)
    m = th.shape[0]
    R = np.zeros(m, np.int32)
    sT = np.zeros((m, 2), np.int64)
    stride = int(sm.max()) if m else 0
    S = np.full((m, stride), np.nan) if want_S else None
    lib().orc_binom2(m, _p(th), _p(sm), seed, n, cut, _p(R), _p(sT), _p(S), stride)
    return R, sT, S


def hier4_posterior(y, n: int = N_PER_ARM) -> np.ndarray:
    """P(p_i > p_0 | y), i = 1..3, of the 4-arm hierarchical model (oracle_hier.c, Section 10.1)."""
    yy = np.ascontiguousarray(y, np.int32)
    P = np.zeros(3)
    lib().orc_hier4_posterior(_p(yy), n, _p(P))
    return P


def hier4_table(idx, n: int = N_PER_ARM) -> np.ndarray:
    """The design statistics 1 - P(p_i > p_0 | y) [len(idx), 3] for outcome indices
    ((y0 m + y1) m + y2) m + y3, m = n + 1 (summed as complements, oracle_hier.c)."""
    ii = np.ascontiguousarray(idx, np.int64)
    out = np.zeros((ii.size, 3))
    lib().orc_hier4_table(n, _p(ii), ii.size, _p(out))
    return out


def sim_hier4(theta_tiles, cfg, sims, seed: int, cut: float, n: int = N_PER_ARM, want_S: bool = False):
    """4-arm design per tile (box centre, null configuration b): R = #{S_b < cut}, sumT [m, 4],
    optionally S_b per simulation (float64) and the outcome index of every simulation."""
    th = np.ascontiguousarray(np.asarray(theta_tiles, np.float64).reshape(-1, 4))
    cf = np.ascontiguousarray(cfg, np.int32)
    sm = np.ascontiguousarray(sims, np.int32)
    m = th.shape[0]
    R = np.zeros(m, np.int32)
    sT = np.zeros((m, 4), np.int64)
    stride = int(sm.max()) if m else 0
    S = np.full((m, stride), np.nan) if want_S else None
    Y = np.full((m, stride), -1, np.int64) if want_S else None
    lib().orc_hier4_sim(m, _p(th), _p(cf), _p(sm), seed, n, cut, _p(R), _p(sT), _p(S), stride, _p(Y))
    return R, sT, S, Y


N_EMBED_P23 = 350   # patients per arm in the embedding of the Phase II/III design (Section 9)


def hier4_summary(y, n):
    """Posterior summary with per-arm sample sizes (oracle_hier.c): dict of P[3], Sc[3] = 1 - P,
    mean[4], var[4] (moment-matched node mixture), dmean[3], dvar[3] of theta_i - theta_0."""
    yy = np.ascontiguousarray(y, np.int32)
    nn = np.ascontiguousarray(n, np.int32)
    out = np.zeros(20)
    lib().orc_hier4_summary(_p(yy), _p(nn), _p(out), None, None)
    return dict(P=out[0:3], Sc=out[3:6], mean=out[6:10], var=out[10:14], dmean=out[14:17], dvar=out[17:20])


def gh16():
    x = np.zeros(16)
    w = np.zeros(16)
    lib().orc_gh16(_p(x), _p(w))
    return x, w


def z95() -> float:
    return float(lib().orc_z95())


def pbest(m, v):
    """P(theta_i is the largest) for independent normal marginals (oracle_phase23.c)."""
    mm = np.ascontiguousarray(m, np.float64)
    vv = np.ascontiguousarray(v, np.float64)
    out = np.zeros(4)
    lib().orc_pbest(_p(mm), _p(vv), _p(out))
    return out


def psucc(md, vd, m0, mi, m_add) -> float:
    return float(lib().orc_psucc(md, vd, m0, mi, m_add))


def sim_phase23(theta_tiles, cfg, sims, seed: int, lam: float, want_S=False, want_info=False,
                want_trace=False):
    """Phase II/III design per tile (box centre, configuration b): R = #{S < lam}, sumY [m, 4],
    sumN [m, 4] (observed counts / sample sizes summed over those simulations), optionally S,
    info [m, stride, 11] (outcome, selected arm, looks, n[4], y[4]) and trace [m, stride, 5, 8]."""
    th = np.ascontiguousarray(np.asarray(theta_tiles, np.float64).reshape(-1, 4))
    cf = np.ascontiguousarray(cfg, np.int32)
    sm = np.ascontiguousarray(sims, np.int32)
    m = th.shape[0]
    R = np.zeros(m, np.int32)
    sY = np.zeros((m, 4), np.int64)
    sN = np.zeros((m, 4), np.int64)
    stride = int(sm.max()) if m else 0
    S = np.full((m, stride), np.nan) if want_S else None
    info = np.full((m, stride, 11), -1, np.int32) if want_info else None
    tr = np.full((m, stride, 5, 8), -1, np.int32) if want_trace else None
    lib().orc_phase23_sim(m, _p(th), _p(cf), _p(sm), seed, lam, _p(R), _p(sY), _p(sN), _p(S), stride,
                          _p(info), _p(tr))
    return dict(R=R, sumY=sY, sumN=sN, S=S, info=info, trace=tr)


# --------------------------------------------------- exponential families
# ------------------------------------------------------------ basket design (Section 10.1)
# The standard-of-care rates p_0a are not given in the paper; Berry et al. (2013), whose design
# the case study follows, use a null response rate of 15% in every basket.  The 85% posterior
# rule rejects arm a when 1 - P(p_a > p_0a | y) < 0.15.
BASKET_P0 = 0.15
BASKET_THETA0 = np.full(4, math.log(BASKET_P0 / (1.0 - BASKET_P0)))
BASKET_CUT = 0.15


def _theta0(theta0):
    return np.ascontiguousarray(BASKET_THETA0 if theta0 is None else theta0, np.float64).reshape(4)


def basket_complement(y, n: int = N_PER_ARM, theta0=None) -> np.ndarray:
    """1 - P(p_a > p_0a | y), a = 0..3, under the hierarchical model on the offsets
    theta_a - theta_0a (Laplace mixture over 90 s2 nodes; pinned in tests/test_oracle_basket.py)."""
    yy = np.ascontiguousarray(y, np.int32)
    out = np.zeros(4)
    lib().orc_basket_complement(_p(yy), n, _p(_theta0(theta0)), _p(out))
    return out


def basket_table(idx, n: int = N_PER_ARM, theta0=None) -> np.ndarray:
    ii = np.ascontiguousarray(idx, np.int64)
    out = np.zeros((ii.size, 4))
    lib().orc_basket_table(n, _p(_theta0(theta0)), _p(ii), ii.size, _p(out))
    return out


def sim_basket(theta_tiles, cfg, sims, seed: int, cut: float = BASKET_CUT, theta0=None, n: int = N_PER_ARM,
               want_S: bool = False):
    """Basket design per tile (centre, configuration b, bit a = H_a): R, sum_rej y, S_b."""
    th = np.ascontiguousarray(theta_tiles, np.float64).reshape(-1, 4)
    cf = np.ascontiguousarray(cfg, np.int32)
    sm = np.ascontiguousarray(sims, np.int32)
    m = th.shape[0]
    R = np.zeros(m, np.int32)
    sT = np.zeros((m, 4), np.int64)
    stride = int(sm.max()) if m else 0
    S = np.full((m, stride), np.nan) if want_S else None
    lib().orc_basket_sim(m, _p(th), _p(cf), _p(sm), seed, n, _p(_theta0(theta0)), cut, _p(R), _p(sT), _p(S),
                         stride)
    return R, sT, S


def basket_subboxes(theta, radii, theta0=None):
    """The basket design's null boundaries theta_a = theta_0a are axis-aligned, so every piece
    box ∩ P(b) is itself a box: each box is cut at the boundaries it straddles, and each piece
    with b != 0 (bit a set when the piece lies in theta_a <= theta_0a) becomes a tile simulated
    at its own centre.  Pieces of a box are listed by b ascending.  Returns a list of
    (box index, b, centre [4], radii [4])."""
    t0 = _theta0(theta0)
    theta = np.asarray(theta, np.float64)
    radii = np.asarray(radii, np.float64)
    out = []
    for i in range(theta.shape[0]):
        parts = []   # per arm: list of (centre, radius, in_null)
        for a in range(4):
            c, r = theta[i, a], radii[i, a]
            lo, hi = c - r, c + r
            if lo < t0[a] < hi:
                parts.append([(0.5 * (lo + t0[a]), 0.5 * (t0[a] - lo), True),
                              (0.5 * (t0[a] + hi), 0.5 * (hi - t0[a]), False)])
            else:
                parts.append([(c, r, hi <= t0[a])])
        pieces = []
        for combo in itertools.product(*parts):
            b = sum(1 << a for a in range(4) if combo[a][2])
            if b:
                pieces.append((b, np.array([x[0] for x in combo]), np.array([x[1] for x in combo])))
        for b, c, r in sorted(pieces, key=lambda q: q[0]):
            out.append((i, b, c, r))
    return out


def log_partition(family: str, theta: np.ndarray, n: int = N_PER_ARM) -> np.ndarray:
    """A(theta) over the last axis: normal location theta^2/2 (Section 4.2);
    independent binomial arms in logit, sum_a n softplus(theta_a) (Example 1)."""
    if family == "normal":
        return 0.5 * np.sum(theta * theta, axis=-1)
    if family == "binom":
        return n * np.sum(np.logaddexp(0.0, theta), axis=-1)
    raise ValueError(family)


def psi(family, theta0, v, q, n=N_PER_ARM):
    """psi(theta0, v, q) = A(theta0 + q v) - A(theta0) for a natural exponential family (Example 1)."""
    return log_partition(family, theta0 + q * v, n) - log_partition(family, theta0, n)


def log_tilt(family, theta0, v, q, a, n=N_PER_ARM):
    """log of the Tilt-Bound U(theta0, v, q, a) (Theorem 1, exponential-family form of Example 1)."""
    return (1.0 - 1.0 / q) * np.log(a) + psi(family, theta0, v, q, n) / q - psi(family, theta0, v, 1.0, n)


def log_inv_tilt(family, theta0, v, q, alpha, n=N_PER_ARM):
    """log of the Inverted Tilt-Bound U^{-1}(theta0, v, q, alpha) (Section 7.2)."""
    return q / (q - 1.0) * (np.log(alpha) - psi(family, theta0, v, q, n) / q + psi(family, theta0, v, 1.0, n))


_GOLD = (math.sqrt(5.0) - 1.0) / 2.0
S_LO, S_HI, GOLD_ITERS = -30.0, 30.0, 100


def _golden(f, m: int, maximize: bool):
    """Golden-section search on s = log(q - 1) in [S_LO, S_HI], vectorised over m problems.

    Valid because the objective is quasi-convex in q (Theorem 2) and q -> log(q-1) is monotone.
    """
    sgn = -1.0 if maximize else 1.0
    lo = np.full(m, S_LO)
    hi = np.full(m, S_HI)
    x1 = hi - _GOLD * (hi - lo)
    x2 = lo + _GOLD * (hi - lo)
    f1 = sgn * f(x1)
    f2 = sgn * f(x2)
    for _ in range(GOLD_ITERS):
        left = f1 <= f2          # the minimum lies in [lo, x2]: drop (x2, hi]
        nlo = np.where(left, lo, x1)
        nhi = np.where(left, x2, hi)
        nx1 = np.where(left, nhi - _GOLD * (nhi - nlo), x2)
        nx2 = np.where(left, x1, nlo + _GOLD * (nhi - nlo))
        fe = sgn * f(np.where(left, nx1, nx2))   # the one new evaluation
        nf1 = np.where(left, fe, f2)
        nf2 = np.where(left, f1, fe)
        lo, hi, x1, x2, f1, f2 = nlo, nhi, nx1, nx2, nf1, nf2
    s = 0.5 * (lo + hi)
    return s, f(s)


def tile_bound(family, theta0, V, a, n=N_PER_ARM):
    """Tilewise Optimized Tilt-Bound inf_q max_{v in V} U(theta0, v, q, a) (Remark 3, Theorem 3).

    theta0 [m, d]; V [m, nv, d] displacements of the tile's vertices from theta0;
    a [m].  Returns (bound [m], q_star [m]).  a == 0 gives 0; a >= 1 gives 1.
    """
    theta0 = np.asarray(theta0, np.float64)
    V = np.asarray(V, np.float64)
    a = np.asarray(a, np.float64)
    m = theta0.shape[0]
    a_safe = np.clip(a, 1e-300, 1.0)
    A0 = log_partition(family, theta0, n)[:, None]                      # [m, 1]
    psi1 = log_partition(family, theta0[:, None, :] + V, n) - A0       # [m, nv]

    def W(s):
        q = (1.0 + np.exp(s))[:, None]                                  # [m, 1]
        psiq = log_partition(family, theta0[:, None, :] + q[:, :, None] * V, n) - A0
        lu = (1.0 - 1.0 / q) * np.log(a_safe)[:, None] + psiq / q - psi1
        return lu.max(axis=1)

    s, w = _golden(W, m, maximize=False)
    with np.errstate(over="ignore"):
        out = np.exp(w)
    out = np.where(a <= 0.0, 0.0, out)
    out = np.where(a >= 1.0, 1.0, np.minimum(out, 1.0))
    return out, 1.0 + np.exp(s)


def tile_inverse(family, theta0, V, alpha, n=N_PER_ARM):
    """alpha' = sup_q min_{v in V} U^{-1}(theta0, v, q, alpha) (Section 7.2).  Returns (alpha', q_star)."""
    theta0 = np.asarray(theta0, np.float64)
    V = np.asarray(V, np.float64)
    m = theta0.shape[0]
    al = np.broadcast_to(np.asarray(alpha, np.float64), (m,))
    A0 = log_partition(family, theta0, n)[:, None]
    psi1 = log_partition(family, theta0[:, None, :] + V, n) - A0

    def W(s):
        q = (1.0 + np.exp(s))[:, None]
        psiq = log_partition(family, theta0[:, None, :] + q[:, :, None] * V, n) - A0
        li = q / (q - 1.0) * (np.log(al)[:, None] - psiq / q + psi1)
        return li.min(axis=1)

    s, w = _golden(W, m, maximize=True)
    return np.exp(w), 1.0 + np.exp(s)


def curvature_bound(family, theta0, radii, n=N_PER_ARM):
    """h_a = sup over the box |theta - theta0| <= r of d^2 A / d theta_a^2: 1 for the normal
    location family, n p(1 - p) at the point of [theta0_a - r_a, theta0_a + r_a] nearest 0 for
    independent binomial arms.  Bounds v' Hess f v by v' Hess A v (reading of Section 4.3's
    f'' <= 1, see taylor_bound)."""
    theta0 = np.asarray(theta0, np.float64)
    r = np.asarray(radii, np.float64)
    if family == "normal":
        return np.ones_like(theta0)
    lo, hi = theta0 - r, theta0 + r
    x = np.where((lo <= 0.0) & (hi >= 0.0), 0.0, np.where(hi < 0.0, hi, lo))
    p = sps.expit(x)
    return n * p * (1.0 - p)


def taylor_bound(family, theta0, radii, V, f, g, n=N_PER_ARM):
    """Second-order Taylor comparison bound over each tile (Section 4.3):
    f(theta0 + v) <= f + g . v + (1/2) sum_a h_a v_a^2 with h = curvature_bound (the remainder
    v' Hess f(xi) v is at most v' Hess A(xi) v for a rejection probability in an exponential
    family).  The right side is convex in v, so its maximum over the tile is at a vertex.
    V [m, nv, d] vertex displacements (NaN rows ignored).  Returns (bound clipped to 1, index of
    the maximising vertex)."""
    theta0 = np.asarray(theta0, np.float64)
    V = np.asarray(V, np.float64)
    h = curvature_bound(family, theta0, radii, n)
    val = (np.asarray(f, np.float64)[:, None] + np.einsum("mvd,md->mv", V, np.asarray(g, np.float64))
           + 0.5 * np.einsum("mvd,md->mv", V * V, h))
    val = np.where(np.isnan(val), -np.inf, val)
    j = np.argmax(val, axis=1)
    return np.minimum(val[np.arange(len(j)), j], 1.0), j


def cp_upper(R, N, delta):
    """Clopper-Pearson (1-delta) upper bound Beta^{-1}(1-delta; R+1, N-R) (Section 6.1); 1 when R == N."""
    R = np.asarray(R, np.float64)
    N = np.asarray(N, np.float64)
    out = np.ones(np.broadcast(R, N).shape)
    ok = R < N
    out[ok] = sps.betaincinv((R + 1.0)[ok] if R.ndim else R + 1.0, (N - R)[ok] if N.ndim else N - R,
                             1.0 - delta)
    return out


def cp_lower(R, N, delta):
    """Clopper-Pearson (1-delta) lower bound Beta^{-1}(delta; R, N-R+1) (Section 6.1); 0 when R == 0."""
    R = np.asarray(R, np.float64)
    N = np.asarray(N, np.float64)
    out = np.zeros(np.broadcast(R, N).shape)
    ok = R > 0
    out[ok] = sps.betaincinv(R[ok] if R.ndim else R, (N - R + 1.0)[ok] if N.ndim else N - R + 1.0, delta)
    return out


def tile_lower(family, theta0, V, b, n=N_PER_ARM):
    """Lower Tilt-Bound over each tile (Remark 2 applied to 1 - F): with b <= f(theta0),
    f(theta0 + v) >= 1 - U(theta0, v, q, 1 - b) for every q, so over the tile
    f >= 1 - inf_q max_v U(theta0, v, q, 1 - b).  Returns (lower bound, q_star)."""
    ub, q = tile_bound(family, theta0, V, 1.0 - np.asarray(b, np.float64), n)
    return 1.0 - ub, q


# ------------------------------------------------------------- the platten
def hypotheses(design: str, d: int):
    """Null hypotheses as half-spaces g . theta <= h (Section 5):
    z-test H0: theta <= 0; multi-arm designs (arm 0 control): H_i: theta_i <= theta_0."""
    if design == "ztest1":
        return [(np.array([1.0]), 0.0)]
    out = []
    for i in range(1, d):
        g = np.zeros(d)
        g[i] = 1.0
        g[0] = -1.0
        out.append((g, 0.0))
    return out


def family_of(design: str) -> str:
    if design == "basket4":
        return "binom"
    return "normal" if design == "ztest1" else "binom"


def n_of(design: str) -> int:
    """Patients per arm of the exponential family the bound is taken in: the Phase II/III
    design is a function of its embedding with 350 potential patients per arm (Section 9)."""
    return N_EMBED_P23 if design == "phase23" else N_PER_ARM


def _enumerate_vertices(G, h, d, tol=1e-12):
    """Vertices of {x : G x <= h} by brute force over d-subsets of active constraints."""
    verts = []
    for idx in itertools.combinations(range(G.shape[0]), d):
        A = G[list(idx)]
        if abs(np.linalg.det(A)) < 1e-12:
            continue
        x = np.linalg.solve(A, h[list(idx)])
        if np.all(G @ x <= h + tol * (1.0 + np.abs(h))):
            if not any(np.allclose(x, y, rtol=0, atol=1e-12) for y in verts):
                verts.append(x)
    return np.array(verts)


def subtiles(design: str, theta, radii, keep_all: bool = False, theta0=None):
    """Split each box into its null-configuration pieces box ∩ P(b) with non-empty interior
    (Section 5, Definition 1).  Returns a list of (box index, b bitmask, vertices [nv, d],
    in_null flag); b bit j-1 is hypothesis j.  With keep_all (single-hypothesis designs only),
    a box that meets no null is kept whole with in_null = False.
    """
    theta = np.asarray(theta, np.float64)
    radii = np.asarray(radii, np.float64)
    if design == "basket4":
        # (box, b, vertices, in_null, centre): the pieces are boxes simulated at their centres
        sgn = np.array(list(itertools.product([-1.0, 1.0], repeat=4)))[:, ::-1]
        return [(i, b, c + sgn * r, True, c) for i, b, c, r in basket_subboxes(theta, radii, theta0)]
    m, d = theta.shape
    hyps = hypotheses(design, d)
    p = len(hyps)
    out = []
    corners_sign = np.array(list(itertools.product([-1.0, 1.0], repeat=d)))
    for i in range(m):
        lo = theta[i] - radii[i]
        hi = theta[i] + radii[i]
        corners = theta[i] + corners_sign * radii[i]
        met = False
        for b in range(1, 1 << p):
            cons = []
            for j, (g, hh) in enumerate(hyps):
                if (b >> j) & 1:
                    cons.append((g, hh))          # g.x <= h
                else:
                    cons.append((-g, -hh))        # closure of the complement: g.x >= h
            vals = [corners @ g - hh for g, hh in cons]
            if any(v.min() >= 0.0 for v in vals):
                continue                           # a constraint holds nowhere inside: no interior
            if all(v.max() <= 0.0 for v in vals):
                out.append((i, b, corners.copy(), True))
                met = True
                continue
            G = np.vstack([np.eye(d), -np.eye(d)] + [g[None, :] for g, _ in cons])
            h = np.concatenate([hi, -lo, [hh for _, hh in cons]])
            V = _enumerate_vertices(G, h, d)
            if V.shape[0] < d + 1:
                continue
            c = V.mean(axis=0)
            if np.all(G @ c < h - 1e-12):
                out.append((i, b, V, True))
                met = True
        if not met and keep_all:
            if p != 1:
                raise ValueError("keep_all is defined for single-hypothesis designs")
            out.append((i, 1, corners.copy(), False))
    return out


def _tile_centres(subs, theta):
    """Simulation point of each tile: the box centre, or the piece's own centre (basket)."""
    return np.array([s[4] if len(s) > 4 else theta[s[0]] for s in subs]).reshape(len(subs), -1)


def _pad_vertices(subs, theta):
    nv = max(len(s[2]) for s in subs)
    d = theta.shape[1]
    V = np.zeros((len(subs), nv, d))
    cen = _tile_centres(subs, theta)
    for t, s in enumerate(subs):
        verts = s[2]
        disp = verts - cen[t]
        V[t, : len(disp)] = disp
        V[t, len(disp):] = disp[0]
    return V


# -------------------------------------------------------------- procedures
def simulate(design: str, theta, sims, seed: int, cut: float = 1.96, want_S: bool = False):
    """Per box: (R, score sums, S) from the design's simulator at the box centre."""
    if design == "ztest1":
        return sim_ztest1(theta, sims, seed, cut, want_S)
    if design == "binom2":
        return sim_binom2(theta, sims, seed, cut, N_PER_ARM, want_S)
    raise ValueError(design)


def score_gradient(design: str, theta, R, score, sims, n: int = N_PER_ARM):
    """Score-function estimate of d TIE / d theta: (sum over rejections of T(x) - R grad A(theta)) / N.

    T(x) is the sufficient statistic of the exponential family (Example 1): for the
    z-test the score sum is already sum Z = sum (X - theta); for binomial arms
    grad_a A = n expit(theta_a)."""
    theta = np.asarray(theta, np.float64)
    N = np.asarray(sims, np.float64)
    if design == "ztest1":
        return (np.asarray(score, np.float64).reshape(-1) / N)[:, None]
    if design == "phase23":   # score already sum (y_obs - n_obs expit theta) over rejections
        return np.asarray(score, np.float64) / N[:, None]
    gA = n * sps.expit(theta)
    return (np.asarray(score, np.float64) - np.asarray(R, np.float64)[:, None] * gA) / N[:, None]


def _tile_simulation(design, theta, sims, subs, seed, cut, want_S, theta0=None):
    """Per-tile (R, score, S) for the tiles `subs`: single-hypothesis designs simulate per box;
    the 4-arm design per (box, b) because its event depends on b."""
    box = np.array([s[0] for s in subs])
    if design == "basket4":
        cfg = np.array([s[1] for s in subs], np.int32)
        R, sT, S = sim_basket(_tile_centres(subs, theta), cfg, np.asarray(sims)[box], seed, cut, theta0,
                              want_S=want_S)
        return R, sT, S
    if design == "hier4":
        cfg = np.array([s[1] for s in subs], np.int32)
        R, sT, S, _ = sim_hier4(theta[box], cfg, np.asarray(sims)[box], seed, cut, want_S=want_S)
        return R, sT, S
    if design == "phase23":
        cfg = np.array([s[1] for s in subs], np.int32)
        o = sim_phase23(theta[box], cfg, np.asarray(sims)[box], seed, cut, want_S=want_S)
        score = o["sumY"] - o["sumN"] * sps.expit(theta[box])
        return o["R"], score, o["S"]
    R, score, S = simulate(design, theta, sims, seed, cut, want_S)
    return R[box], score[box], (S[box] if S is not None else None)


def validate(design: str, theta, radii, sims, seed: int, delta: float, cut: float = 1.96,
             keep_all: bool = False, theta0=None):
    """Validation (Algorithm 1): per sub-tile R, CP upper bound, tilewise optimized Tilt-Bound."""
    theta = np.asarray(theta, np.float64)
    subs = subtiles(design, theta, radii, keep_all, theta0)
    box = np.array([s[0] for s in subs])
    N = np.asarray(sims)[box]
    Rb, score, _ = _tile_simulation(design, theta, sims, subs, seed, cut, False, theta0)
    cp = cp_upper(Rb, N, delta)
    V = _pad_vertices(subs, theta)
    cen = _tile_centres(subs, theta)
    ub, qs = tile_bound(family_of(design), cen, V, cp, n=n_of(design))
    cpl = cp_lower(Rb, N, delta)
    lb, _ = tile_lower(family_of(design), cen, V, cpl, n=n_of(design))
    out = dict(box=box, b=np.array([s[1] for s in subs]), R=Rb, N=N, cp=cp, bound=ub,
               q=qs, score=score, subs=subs, cp_lower=cpl, lower=lb)
    if design not in ("hier4", "phase23", "basket4"):
        R, sc, _ = simulate(design, theta, sims, seed, cut)
        out.update(R_box=R, score_box=sc)
    return out


def order_statistic(S_row: np.ndarray, k: int) -> float:
    """k-th smallest value (1-based) of S_row; -inf when k == 0 (no rejection, Theorem 4's range)."""
    if k <= 0:
        return -math.inf
    return float(np.sort(S_row)[k - 1])


def tiebreak_u(seed: int, n: int) -> np.ndarray:
    """The uniform adjoined to each simulation by the randomised test (discussion of Theorem
    (pointwise calibration), Section 7.1): u_k = first word of Philox4x32-10 at counter
    (0, k, 1, 0) with the seed as key, as an integer in [0, 2^32); P(u < c) = c / 2^32.  It is
    disjoint from the data words (counter word 2 = 0) and shared by all tiles."""
    out = np.zeros(max(int(n), 0), np.uint32)
    if n > 0:
        lib().orc_tiebreak_u(seed, int(n), _p(out))
    return out


def order_statistic_pair(S_row: np.ndarray, u_row: np.ndarray, k: int):
    """k-th smallest pair (S, u) in lexicographic order (1-based); (-inf, 0) when k == 0."""
    if k <= 0:
        return -math.inf, 0
    idx = np.lexsort((u_row, S_row))   # primary key S, secondary u
    j = idx[k - 1]
    return float(S_row[j]), int(u_row[j])


def calibrate(design: str, theta, radii, sims, seed: int, alpha: float, keep_all: bool = False,
              key_dtype=np.float64, cut: float = 1.96, theta0=None):
    """Calibration (Algorithm 2): alpha'_i, k_i = floor((N_i+1) alpha'_i), lambda*_i = S_(k_i),
    lambda* = min_i lambda*_i, and #{S < lambda*_i} per sub-tile.  key_dtype=np.float32 takes the
    order statistic and the comparisons in float32 (the precision in which the GPU compares
    the 4-arm statistic)."""
    theta = np.asarray(theta, np.float64)
    sims = np.asarray(sims, np.int32)
    subs = subtiles(design, theta, radii, keep_all, theta0)
    box = np.array([s[0] for s in subs])
    V = _pad_vertices(subs, theta)
    ap, qs = tile_inverse(family_of(design), _tile_centres(subs, theta), V, alpha, n=n_of(design))
    N = sims[box]
    k = np.floor((N + 1.0) * ap).astype(np.int64)
    _, _, S = _tile_simulation(design, theta, sims, subs, seed, cut, True, theta0)
    lam = np.empty(len(subs))
    rej = np.empty(len(subs), np.int64)
    for t in range(len(subs)):
        row = S[t, : N[t]].astype(key_dtype)
        lam[t] = order_statistic(row, int(k[t]))
        rej[t] = int(np.sum(row < key_dtype(lam[t])))   # #{S < lambda*_i}, also for lambda*_i = +inf
    in_null = np.array([bool(s[3]) for s in subs], bool)
    # lambda* = min over the tiles covering the null space (Section 7.3); boxes kept outside it
    # (keep_all) have no Type I Error to control
    return dict(box=box, b=np.array([s[1] for s in subs]), alpha_prime=ap, q=qs, k=k,
                lam=lam, lam_global=float(lam[in_null].min()) if in_null.any() else math.inf,
                reject_at_lam=rej, N=N, subs=subs)


def calibrate_tiebreak(design: str, theta, radii, sims, seed: int, alpha: float, keep_all: bool = False,
                       key_dtype=np.float64, cut: float = 1.96, theta0=None):
    """Randomised calibration: the statistic becomes the pair (S, u) with u from tiebreak_u and
    the threshold the pair (lambda, c), both compared lexicographically.  Per tile: alpha'_i and
    k_i as in calibrate, (lambda_i, c_i) = the k_i-th smallest pair, and the number of pairs
    strictly below it; globally the lexicographic minimum of (lambda_i, c_i)."""
    theta = np.asarray(theta, np.float64)
    sims = np.asarray(sims, np.int32)
    subs = subtiles(design, theta, radii, keep_all, theta0)
    box = np.array([s[0] for s in subs])
    V = _pad_vertices(subs, theta)
    ap, _ = tile_inverse(family_of(design), _tile_centres(subs, theta), V, alpha, n=n_of(design))
    N = sims[box]
    k = np.floor((N + 1.0) * ap).astype(np.int64)
    _, _, S = _tile_simulation(design, theta, sims, subs, seed, cut, True, theta0)
    u = tiebreak_u(seed, int(N.max()) if len(N) else 0)
    lam = np.empty(len(subs))
    c = np.zeros(len(subs), np.int64)
    rej = np.zeros(len(subs), np.int64)
    for t in range(len(subs)):
        row = S[t, : N[t]].astype(key_dtype)
        ur = u[: N[t]]
        lam[t], c[t] = order_statistic_pair(row, ur, int(k[t]))
        if k[t] > 0:
            L = key_dtype(lam[t])
            rej[t] = int(np.sum(row < L) + np.sum((row == L) & (ur < c[t])))
    in_null = np.flatnonzero([bool(s[3]) for s in subs])   # the minimum runs over the null space
    g = int(in_null[np.lexsort((c[in_null], lam[in_null]))[0]]) if len(in_null) else -1
    return dict(box=box, b=np.array([s[1] for s in subs]), alpha_prime=ap, k=k, lam=lam, c=c,
                reject_at=rej, lam_global=float(lam[g]) if g >= 0 else math.inf,
                c_global=int(c[g]) if g >= 0 else 0, N=N, subs=subs)


# ---------------------------------------------------- confidence sets (Section 8)
def estimand_range(subs, coef, link: str = "linear"):
    """Range of e over each tile (Section 8's image of a tile under e):
    e(theta) = c0 + sum_a c_a g(theta_a), coef = (c_1 .. c_d, c0), g the identity ("linear")
    or expit ("expit", e.g. p_1 - p_0).  Linear: min / max over the tile's vertices (exact on a
    polytope).  Expit: the sum over coordinates of the extremes of c_a expit(theta_a) over the
    tile's bounding box (exact on a box, an enclosing interval on a clipped tile)."""
    coef = np.asarray(coef, np.float64)
    c, c0 = coef[:-1], coef[-1]
    lo = np.empty(len(subs))
    hi = np.empty(len(subs))
    for t, s in enumerate(subs):
        V = np.asarray(s[2], np.float64)
        if link == "linear":
            vals = V @ c + c0
            lo[t], hi[t] = vals.min(), vals.max()
        elif link == "expit":
            a = c * sps.expit(V.min(axis=0))
            b = c * sps.expit(V.max(axis=0))
            lo[t] = c0 + np.minimum(a, b).sum()
            hi[t] = c0 + np.maximum(a, b).sum()
        else:
            raise ValueError(link)
    return lo, hi


def confidence_set(subs, lam, s_obs, coef, link: str = "linear", key_dtype=np.float32):
    """Section 8: with the observed statistic s_i of each tile and its calibrated threshold
    lambda_i, the confidence region is the union of the tiles not rejected, s_i >= lambda_i
    (the test rejects when s_i < lambda_i; compared in key_dtype, the precision of the
    simulated statistic), and the confidence set of e is the image of that region: returns
    (keep mask, per-tile range (lo, hi), (min lo, max hi) over kept tiles, or (+inf, -inf)
    when none is kept)."""
    sk = np.broadcast_to(np.asarray(s_obs, np.float64).astype(key_dtype), (len(subs),))
    keep = ~(sk < np.asarray(lam, np.float64).astype(key_dtype))
    lo, hi = estimand_range(subs, coef, link)
    rng = (float(lo[keep].min()), float(hi[keep].max())) if keep.any() else (math.inf, -math.inf)
    return keep, lo, hi, rng
