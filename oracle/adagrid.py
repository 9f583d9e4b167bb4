"""CPU ORACLE -- test infrastructure only (see the package header): adaptive gridding and
simulation allocation from pilot runs, for validation and for calibration.

The paper states the goal and the outcome only (Section 10.2, the Phase II/III calibration:
pilot simulations choose the tiles' geometry and simulation counts, from 2,048 to 524,288
simulations per tile and half-widths from 0.0625 down to 0.000488).  The rule below is this
package's reading of it, written out plainly:

Validation (Algorithm 1 per round).  For each box, over its tiles: U = max tile bound,
geometric part G = max(bound - cp_upper) (what a smaller tile removes), Monte Carlo part
M = max(cp_upper - R/N) (what more simulations remove).  A box with U <= target is done;
otherwise it is split into 2^d children of half the half-width when G >= M and the children
stay >= r_min, else its N doubles when 2N <= n_max, else it splits if it can, else it is
stuck (code 3: the target is out of reach within the limits).

Calibration (Algorithm 2 per round).  lambda* = min over all tiles.  A box is critical when
its smallest lambda_i <= lambda* + margin.  For the tile giving that smallest lambda_i: the
geometric slack alpha - alpha'_i against the spread of the calibrated level, the standard
deviation sqrt(alpha'(1 - alpha')/(N + 2)) of f(lambda_hat) ~ Beta(k, N - k + 1)
(Theorem 4).  Split when the slack is at least that spread (and the children stay >= r_min),
else double N (<= n_max), else split if possible, else stuck.  Boxes that are not critical
are left as they are, but are re-examined every round (lambda* moves).

Every round re-simulates only the boxes that changed (children or doubled N), with the same
seed: under common random numbers a box's first N simulations are the same draws after its
N doubles.  Children of a box replace it in place, in the order c = 0 .. 2^d - 1 with
coordinate a in the upper half when bit a of c is set.
"""
from __future__ import annotations

import math

import numpy as np

from . import (calibrate, subtiles, validate)

DONE, SPLIT, DOUBLE, STUCK = 0, 1, 2, 3


def split_box(theta, radii):
    """The 2^d children of one box: half the half-width, centres at theta +- r/2."""
    theta = np.asarray(theta, np.float64)
    radii = np.asarray(radii, np.float64)
    d = theta.size
    kids = []
    for c in range(1 << d):
        sgn = np.array([1.0 if (c >> a) & 1 else -1.0 for a in range(d)])
        kids.append((theta + sgn * radii / 2.0, radii / 2.0))
    return kids


def _per_box(n_boxes, box_of_tile, values, reduce):
    out = [None] * n_boxes
    for t, b in enumerate(box_of_tile):
        out[b] = values[t] if out[b] is None else reduce(out[b], values[t])
    return out


def decide_validation(radii, sims, box_of_tile, bound, cp, fhat, target, r_min, n_max):
    """Per-box decision codes of the validation rule (module header)."""
    n = len(sims)
    U = _per_box(n, box_of_tile, bound, max)
    G = _per_box(n, box_of_tile, np.asarray(bound) - np.asarray(cp), max)
    M = _per_box(n, box_of_tile, np.asarray(cp) - np.asarray(fhat), max)
    dec = np.zeros(n, np.int32)
    for i in range(n):
        if U[i] is None or U[i] <= target:
            continue
        can_split = np.min(radii[i]) / 2.0 >= r_min
        can_double = 2 * int(sims[i]) <= n_max
        if G[i] >= M[i] and can_split:
            dec[i] = SPLIT
        elif can_double:
            dec[i] = DOUBLE
        elif can_split:
            dec[i] = SPLIT
        else:
            dec[i] = STUCK
    return dec


def decide_calibration(radii, sims, box_of_tile, lam, alpha_prime, N, alpha, margin, r_min, n_max):
    """Per-box decision codes of the calibration rule (module header)."""
    n = len(sims)
    lam = np.asarray(lam, np.float64)
    lam_star = lam.min() if len(lam) else math.inf
    best = [None] * n                      # tile with the box's smallest lambda (first on ties)
    for t, b in enumerate(box_of_tile):
        if best[b] is None or lam[t] < lam[best[b]]:
            best[b] = t
    thr = lam_star + margin
    if math.isnan(thr):                    # lambda* = -inf with an infinite margin: every box
        thr = math.inf
    dec = np.zeros(n, np.int32)
    for i in range(n):
        t = best[i]
        if t is None or not lam[t] <= thr:
            continue
        ap = float(alpha_prime[t])
        slack = alpha - ap
        spread = math.sqrt(max(ap * (1.0 - ap), 0.0) / (float(N[t]) + 2.0))
        can_split = np.min(radii[i]) / 2.0 >= r_min
        can_double = 2 * int(sims[i]) <= n_max
        if slack >= spread and can_split:
            dec[i] = SPLIT
        elif can_double:
            dec[i] = DOUBLE
        elif can_split:
            dec[i] = SPLIT
        else:
            dec[i] = STUCK
    return dec


def apply(theta, radii, sims, dec):
    """New box list: split boxes replaced in place by their children, doubled boxes with 2N.
    Returns (theta, radii, sims, parent index, changed mask)."""
    th, rd, sm, par, ch = [], [], [], [], []
    for i in range(len(sims)):
        if dec[i] == SPLIT:
            for ct, cr in split_box(theta[i], radii[i]):
                th.append(ct)
                rd.append(cr)
                sm.append(int(sims[i]))
                par.append(i)
                ch.append(True)
        else:
            th.append(np.asarray(theta[i], np.float64))
            rd.append(np.asarray(radii[i], np.float64))
            sm.append(int(sims[i]) * (2 if dec[i] == DOUBLE else 1))
            par.append(i)
            ch.append(dec[i] == DOUBLE)
    d = np.asarray(theta).shape[1]
    return (np.array(th).reshape(-1, d), np.array(rd).reshape(-1, d), np.array(sm, np.int32),
            np.array(par, np.int64), np.array(ch, bool))


def _box_tiles(design, theta, radii, keep_all):
    subs = subtiles(design, theta, radii, keep_all)
    return subs, np.array([s[0] for s in subs], np.int64)


def run(design, theta, radii, sims, seed, mode="validate", target=0.03, alpha=0.025, delta=0.01,
        margin=0.0, r_min=0.0, n_max=1 << 20, max_rounds=8, keep_all=False, cut=1.96, key_dtype=np.float64):
    """Adaptive rounds (module header).  Per round the simulated boxes are only those that
    changed; their per-tile results are kept with the box.  Returns the final boxes, their
    tiles' results, and per-round (n_boxes, n_split, n_double, n_stuck, sims simulated)."""
    theta = np.asarray(theta, np.float64).copy()
    radii = np.asarray(radii, np.float64).copy()
    sims = np.asarray(sims, np.int32).copy()
    store = [None] * len(sims)             # per box: dict of its tiles' results
    changed = np.ones(len(sims), bool)
    history = []
    for rnd in range(max_rounds + 1):
        idx = np.flatnonzero(changed)
        simulated = 0
        if len(idx):
            th, rd, sm = theta[idx], radii[idx], sims[idx]
            subs, tb = _box_tiles(design, th, rd, keep_all)
            for j in range(len(idx)):
                store[idx[j]] = None
            if len(subs):
                if mode == "validate":
                    o = validate(design, th, rd, sm, seed, delta, cut=cut, keep_all=keep_all)
                    per = dict(bound=o["bound"], cp=o["cp"], fhat=o["R"] / o["N"], R=o["R"], N=o["N"])
                else:
                    o = calibrate(design, th, rd, sm, seed, alpha, keep_all=keep_all, key_dtype=key_dtype,
                                  cut=cut)
                    per = dict(lam=o["lam"], alpha_prime=o["alpha_prime"], k=o["k"], N=o["N"])
                for j in range(len(idx)):
                    sel = tb == j
                    store[idx[j]] = {k: v[sel] for k, v in per.items()}
                simulated = int(np.sum(sm[np.unique(tb)]))
        # flatten the stored results in box order
        box_of_tile = np.concatenate([np.full(len(next(iter(s.values()))), i, np.int64)
                                      for i, s in enumerate(store) if s is not None] or [np.zeros(0, np.int64)])
        cat = {}
        keys = ("bound", "cp", "fhat", "R", "N") if mode == "validate" else ("lam", "alpha_prime", "k", "N")
        for k in keys:
            cat[k] = np.concatenate([s[k] for s in store if s is not None] or [np.zeros(0)])
        if mode == "validate":
            dec = decide_validation(radii, sims, box_of_tile, cat["bound"], cat["cp"], cat["fhat"], target,
                                    r_min, n_max)
        else:
            dec = decide_calibration(radii, sims, box_of_tile, cat["lam"], cat["alpha_prime"], cat["N"], alpha,
                                     margin, r_min, n_max)
        history.append((len(sims), int(np.sum(dec == SPLIT)), int(np.sum(dec == DOUBLE)),
                        int(np.sum(dec == STUCK)), simulated))
        if rnd == max_rounds or not np.any((dec == SPLIT) | (dec == DOUBLE)):
            return dict(theta=theta, radii=radii, sims=sims, decision=dec, box_of_tile=box_of_tile,
                        tiles=cat, history=history, rounds=rnd)
        theta, radii, sims, par, changed = apply(theta, radii, sims, dec)
        store = [None if changed[i] else store[par[i]] for i in range(len(sims))]
