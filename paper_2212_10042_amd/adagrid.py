"""Adaptive gridding and simulation allocation from pilot runs (Section 10.2 reports its
Phase II/III calibration on tiles and simulation counts chosen this way).

Rounds of: the GPU pass (cse_validate, or cse_calibrate) over the boxes that changed, the
library's host decision step (cse_adagrid_decide, then cse_adagrid_apply: split into 2^d
children, double N, done or stuck; the rule is documented with those calls in cse.h), and a
checkpoint of the whole state (boxes, the results of every box's tiles, the round, the
history) written atomically to an .npz file, from which `run(..., resume=True)` continues.

Boxes that did not change keep their tiles' results: with the same seed and common random
numbers, simulating them again would reproduce the same values, and a doubled box's first N
simulations are the same draws as before.
"""
from __future__ import annotations

import json
import os

import numpy as np
import torch

from . import (CSE_EINVAL, CseError, Platten, cse_adagrid_apply, cse_adagrid_decide,
               cse_adagrid_rule)

DONE, SPLIT, DOUBLE, STUCK = 0, 1, 2, 3
_TILE_KEYS = {"validate": ("a", "b", "c", "R", "N"), "calibrate": ("a", "b", "c", "k")}


def _pass(kind, mode, theta, radii, sims, seed, alpha, delta, keep_all, cut):
    """One GPU pass over the given boxes: per-tile (box index within them, a, b, c, extra)."""
    try:
        P = Platten.create(kind, theta, radii, sims, cut=cut, keep_all=keep_all)
    except CseError as e:
        if e.status == CSE_EINVAL and "no box meets the null" in str(e):
            return None
        raise
    try:
        box = np.asarray(P.tiles["box"], np.int64)
        N = np.asarray(sims, np.float64)[box]
        if mode == "validate":
            o = P.validate(seed, delta=delta)
            torch.cuda.synchronize()
            R = o["reject"].cpu().numpy().astype(np.float64)
            out = dict(box=box, a=o["tile_bound"].cpu().numpy(), b=o["cp_upper"].cpu().numpy(), c=R / N, R=R, N=N)
        else:
            o = P.calibrate(seed, alpha=alpha, with_validation=False)
            torch.cuda.synchronize()
            out = dict(box=box, a=o["lambda_tile"].cpu().numpy(), b=o["alpha_prime"].cpu().numpy(), c=N,
                       k=o["k"].cpu().numpy().astype(np.float64))
    finally:
        P.close()
    return out


def _save(path, st):
    tmp = path + ".tmp.npz"
    np.savez(tmp, **{k: v for k, v in st.items() if k not in ("meta", "history")},
             meta=np.array(json.dumps(st["meta"])), history=np.array(st["history"], np.int64).reshape(-1, 5))
    os.replace(tmp, path)


def _load(path):
    with np.load(path, allow_pickle=False) as z:
        st = {k: z[k] for k in z.files}
    st["meta"] = json.loads(str(st["meta"]))
    st["history"] = [tuple(int(x) for x in h) for h in st["history"]]
    st["round"] = int(st["round"])
    return st


def run(kind, theta, radii, sims, seed, mode="validate", target=0.03, alpha=0.025, delta=0.01, margin=0.0,
        r_min=0.0, n_max=1 << 20, max_rounds=8, keep_all=False, cut=None, checkpoint=None, resume=False,
        on_round=None):
    """Adaptive rounds until no box splits or doubles, or max_rounds.  Returns the final boxes
    (theta, radii, sims), the last decisions, the tiles' results in box order (tile_box and
    the arrays a, b, c: validation bound, cp_upper, R/N; calibration lambda, alpha', N) and
    per-round (n_boxes, splits, doubles, stuck, simulations run)."""
    if mode not in _TILE_KEYS:
        raise ValueError("mode is 'validate' or 'calibrate'")
    meta = dict(kind=kind, mode=mode, target=target, alpha=alpha, delta=delta, margin=margin, r_min=r_min,
                n_max=int(n_max), seed=int(seed), keep_all=bool(keep_all), cut=cut)
    keys = _TILE_KEYS[mode]
    if resume and checkpoint and os.path.exists(checkpoint):
        st = _load(checkpoint)
        if st["meta"] != meta:
            raise ValueError(f"checkpoint {checkpoint} was made with other settings: {st['meta']}")
    else:
        th = np.ascontiguousarray(theta, np.float64)
        st = dict(theta=th, radii=np.ascontiguousarray(radii, np.float64), sims=np.ascontiguousarray(sims, np.int32),
                  changed=np.ones(len(sims), bool), tile_box=np.zeros(0, np.int64), round=0, history=[], meta=meta)
        for k in keys:
            st["t_" + k] = np.zeros(0)
    d = st["theta"].shape[1]
    rule = cse_adagrid_rule(mode=0 if mode == "validate" else 1, d=d, target=target, alpha=alpha, margin=margin,
                            r_min=r_min, n_max=int(n_max))
    while True:
        idx = np.flatnonzero(st["changed"])
        simulated = 0
        if len(idx):
            o = _pass(kind, mode, st["theta"][idx], st["radii"][idx], st["sims"][idx], seed, alpha, delta,
                      keep_all, cut)
            if o is not None:
                gb = idx[o["box"]]
                simulated = int(st["sims"][idx][np.unique(o["box"])].sum())
                tb = np.concatenate([st["tile_box"], gb])
                cols = {k: np.concatenate([st["t_" + k], o[k]]) for k in keys}
                order = np.argsort(tb, kind="stable")
                st["tile_box"] = tb[order]
                for k in keys:
                    st["t_" + k] = cols[k][order]
            st["changed"][:] = False
        dec = cse_adagrid_decide(rule, st["radii"], st["sims"], st["tile_box"], st["t_a"], st["t_b"], st["t_c"])
        if len(st["history"]) <= st["round"]:   # not already recorded (a resumed final checkpoint is)
            st["history"].append((len(st["sims"]), int(np.sum(dec == SPLIT)), int(np.sum(dec == DOUBLE)),
                                  int(np.sum(dec == STUCK)), simulated))
            if on_round:
                on_round(st["round"], st["history"][-1])
        if st["round"] >= max_rounds or not np.any((dec == SPLIT) | (dec == DOUBLE)):
            st["decision"] = dec
            if checkpoint:
                _save(checkpoint, st)
            res = dict(theta=st["theta"], radii=st["radii"], sims=st["sims"], decision=dec, tile_box=st["tile_box"],
                       history=st["history"], rounds=st["round"])
            res.update({k: st["t_" + k] for k in keys})
            return res
        th, rd, sm, par, ch = cse_adagrid_apply(st["theta"], st["radii"], st["sims"], dec)
        # tiles of boxes that did not change move to their new index; the others are dropped
        new_of_old = np.full(len(st["sims"]), -1, np.int64)
        keep_new = np.flatnonzero(~ch)
        new_of_old[par[keep_new]] = keep_new
        nb = new_of_old[st["tile_box"]]
        kept = nb >= 0
        st["tile_box"] = nb[kept]
        for k in keys:
            st["t_" + k] = st["t_" + k][kept]
        st.update(theta=th, radii=rd, sims=sm, changed=ch, round=st["round"] + 1)
        if checkpoint:
            _save(checkpoint, st)
