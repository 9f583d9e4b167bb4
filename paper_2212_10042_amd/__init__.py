"""Continuous Simulation Extension on MI355X (gfx950): Python binding of libcse.so.

The functions named ``cse_*`` marshal arguments to the C ABI of the same name
(include/cse.h): torch tensors supply device memory and the current HIP stream,
every computation runs in the library's HIP kernels.  If libcse.so is missing the
import fails; there is no other execution path.

Method: Yang, Thompson & Sklar, "Guarantees for Comprehensive Simulation
Assessment of Statistical Methods" -- validation (Algorithm 1, Section 6) and
calibration (Algorithm 2, Section 7) over a platten of tiles (Definition 1,
Section 5), with the Tilt-Bound of Theorem 1.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcse.so")

CSE_OK, CSE_EINVAL, CSE_ENOMEM, CSE_EHIP, CSE_EUNSUPPORTED, CSE_ECALIB = 0, -1, -2, -3, -4, -5
CSE_ZTEST1, CSE_BINOM2_Z, CSE_HIER4, CSE_PHASE23, CSE_BASKET4 = 1, 2, 3, 4, 5
BASKET_P0 = 0.15   # standard-of-care rate of every basket unless given (not stated in the paper)
CSE_PLATTEN_KEEP_ALL = 1

EXPORTED = ("cse_platten_create", "cse_platten_destroy", "cse_platten_size", "cse_platten_describe",
            "cse_simulate", "cse_validate", "cse_calibrate", "cse_bound", "cse_simulate_per_tile",
            "cse_platten_stats", "cse_profile_enable", "cse_profile_get", "cse_profile_reset",
            "cse_posterior_table", "cse_work_counters", "cse_plan_validate", "cse_plan_calibrate",
            "cse_plan_launch", "cse_plan_nodes", "cse_plan_destroy", "cse_autotune", "cse_taylor",
            "cse_validate_lower", "cse_confidence_set", "cse_calibrate_tiebreak", "cse_adagrid_decide",
            "cse_adagrid_apply", "cse_platten_tiles", "cse_calibrate_noalloc", "cse_platten_set_option",
            "cse_last_error")


class CseError(RuntimeError):
    def __init__(self, fn: str, status: int, msg: str):
        super().__init__(f"{fn} -> status {status}: {msg}")
        self.status = status


class cse_adagrid_rule(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("d", ctypes.c_int32), ("target", ctypes.c_double),
                ("alpha", ctypes.c_double), ("margin", ctypes.c_double), ("r_min", ctypes.c_double),
                ("n_max", ctypes.c_int64)]


class cse_design(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("n_arms", ctypes.c_int32), ("n_per_arm", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("cut", ctypes.c_double), ("theta0", ctypes.c_double * 4)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built (python -m paper_2212_10042_amd.build)")
    L = ctypes.CDLL(LIB_PATH)
    missing = [fn for fn in EXPORTED if not hasattr(L, fn)]
    if missing:
        raise ImportError(f"{LIB_PATH} is stale (missing {missing}); rebuild it")
    P, i32, i64, u64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_double
    L.cse_platten_create.argtypes = [ctypes.POINTER(cse_design), i64, P, P, P, i32, ctypes.POINTER(P)]
    L.cse_platten_destroy.argtypes = [P]
    L.cse_platten_size.argtypes = [P]
    L.cse_platten_size.restype = i64
    L.cse_platten_describe.argtypes = [P, P, P, P, P]
    L.cse_platten_tiles.argtypes = [P, P, P]
    L.cse_simulate.argtypes = [P, u64, P, P, P, P, P]
    L.cse_validate.argtypes = [P, u64, dbl, P, P, P, P, P, P, P, P]
    L.cse_calibrate.argtypes = [P, u64, dbl, P, P, P, P, P, dbl, P, P, P, P, P, P, P]
    L.cse_calibrate_noalloc.argtypes = [P, u64, dbl, P, P, P, P, P, dbl, P, P, P, P, P, P, P]
    L.cse_bound.argtypes = [P, i32, P, P, dbl, P, P, P]
    L.cse_simulate_per_tile.argtypes = [P, u64, i64, i64, P, P]
    L.cse_platten_stats.argtypes = [P, P]
    L.cse_posterior_table.argtypes = [P, P, i64, ctypes.POINTER(i64), P]
    L.cse_work_counters.argtypes = [P, P, P]
    L.cse_platten_set_option.argtypes = [P, i32, dbl]
    L.cse_plan_validate.argtypes = [P, u64, dbl] + [P] * 7 + [ctypes.POINTER(P)]
    L.cse_plan_calibrate.argtypes = [P, u64, dbl, P, P, P, P, P, dbl] + [P] * 6 + [ctypes.POINTER(P)]
    L.cse_plan_launch.argtypes = [P, P]
    L.cse_plan_nodes.argtypes = [P]
    L.cse_plan_nodes.restype = i64
    L.cse_plan_destroy.argtypes = [P]
    L.cse_autotune.argtypes = [P, u64, i64, P, P]
    L.cse_taylor.argtypes = [P, P, P, P, P, P, P]
    L.cse_validate_lower.argtypes = [P, P, dbl, P, P, P, P]
    L.cse_adagrid_decide.argtypes = [ctypes.POINTER(cse_adagrid_rule), i64, P, P, i64, P, P, P, P, P]
    L.cse_adagrid_apply.argtypes = [i32, i64, P, P, P, P, i64, P, P, P, P, P, ctypes.POINTER(i64)]
    L.cse_confidence_set.argtypes = [P, P, i64, P, P, i32, P, P, P, P, P]
    L.cse_calibrate_tiebreak.argtypes = [P, u64, dbl] + [P] * 8
    L.cse_profile_enable.argtypes = [i32]
    L.cse_profile_get.argtypes = [ctypes.c_char_p, ctypes.POINTER(i64), ctypes.POINTER(dbl)]
    L.cse_profile_reset.argtypes = []
    L.cse_last_error.restype = ctypes.c_char_p
    for fn in EXPORTED:
        if fn not in ("cse_platten_size", "cse_last_error", "cse_plan_nodes"):
            getattr(L, fn).restype = ctypes.c_int
    return L


_L = _load()


def lib():
    return _L


def _check(fn: str, status: int):
    if status != CSE_OK:
        raise CseError(fn, status, _L.cse_last_error().decode())


def _ptr(t):
    if t is None:
        return None
    if isinstance(t, torch.Tensor):
        return ctypes.c_void_p(t.data_ptr())
    if isinstance(t, np.ndarray):
        return t.ctypes.data_as(ctypes.c_void_p)
    raise TypeError(type(t))


def _stream(stream=None):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


# ------------------------------------------------------------------ C-ABI mirrors
def make_design(kind: str | int, cut: float | None = None, n_per_arm: int | None = None,
                theta0=None) -> cse_design:
    """Design descriptor.  cut defaults: 1.96 (z designs), 0.05 (4-arm hierarchical),
    0.06253 (Phase II/III final-analysis lambda), 0.15 (basket: the 85% rule); n_per_arm: 35,
    or the embedding's 350; theta0 (basket): logit of each arm's fixed rate, default
    logit(0.15) for every arm."""
    k = {"ztest1": CSE_ZTEST1, "binom2": CSE_BINOM2_Z, "hier4": CSE_HIER4, "phase23": CSE_PHASE23,
         "basket4": CSE_BASKET4}.get(kind, kind)
    d = {CSE_ZTEST1: 1, CSE_BINOM2_Z: 2, CSE_HIER4: 4, CSE_PHASE23: 4, CSE_BASKET4: 4}[k]
    if cut is None:
        cut = {CSE_ZTEST1: 1.96, CSE_BINOM2_Z: 1.96, CSE_HIER4: 0.05, CSE_PHASE23: 0.06253, CSE_BASKET4: 0.15}[k]
    if n_per_arm is None:
        n_per_arm = 0 if k == CSE_ZTEST1 else (350 if k == CSE_PHASE23 else 35)
    t0 = np.zeros(4)
    if k == CSE_BASKET4:
        t0 = np.full(4, np.log(BASKET_P0 / (1 - BASKET_P0))) if theta0 is None else np.asarray(theta0, np.float64)
    return cse_design(k, d, n_per_arm, 0, float(cut), (ctypes.c_double * 4)(*[float(x) for x in t0]))


def cse_platten_tiles(h, n_tiles: int, d: int):
    """Host copies of every tile's simulation point and half-widths."""
    th = np.zeros((n_tiles, d))
    rd = np.zeros((n_tiles, d))
    _check("cse_platten_tiles", _L.cse_platten_tiles(h, _ptr(th), _ptr(rd)))
    return th, rd


def cse_platten_create(design: cse_design, theta, radii, sims, flags: int = 0):
    th = np.ascontiguousarray(theta, np.float64)
    rd = np.ascontiguousarray(radii, np.float64)
    sm = np.ascontiguousarray(sims, np.int32)
    h = ctypes.c_void_p()
    _check("cse_platten_create",
           _L.cse_platten_create(ctypes.byref(design), th.shape[0], _ptr(th), _ptr(rd), _ptr(sm),
                                 flags, ctypes.byref(h)))
    return h


def cse_platten_destroy(h):
    _check("cse_platten_destroy", _L.cse_platten_destroy(h))


def cse_platten_size(h) -> int:
    return int(_L.cse_platten_size(h))


def cse_platten_describe(h):
    n = cse_platten_size(h)
    box = np.zeros(n, np.int64)
    cfg = np.zeros(n, np.int32)
    nv = np.zeros(n, np.int32)
    inn = np.zeros(n, np.int32)
    _check("cse_platten_describe", _L.cse_platten_describe(h, _ptr(box), _ptr(cfg), _ptr(nv), _ptr(inn)))
    return dict(box=box, cfg=cfg, n_vert=nv, in_null=inn)


def cse_simulate(h, seed, reject, score_T=None, score_Z=None, grad=None, stream=None):
    _check("cse_simulate", _L.cse_simulate(h, seed, _ptr(reject), _ptr(score_T), _ptr(score_Z),
                                           _ptr(grad), _stream(stream)))


def cse_validate(h, seed, delta, reject, score_T, score_Z, grad, cp_upper, tile_bound, q_star=None,
                 stream=None):
    _check("cse_validate", _L.cse_validate(h, seed, delta, _ptr(reject), _ptr(score_T), _ptr(score_Z),
                                           _ptr(grad), _ptr(cp_upper), _ptr(tile_bound), _ptr(q_star),
                                           _stream(stream)))


def cse_calibrate(h, seed, alpha, alpha_prime, k, lambda_tile, lambda_global, reject_at_lambda=None,
                  delta=0.01, reject=None, score_T=None, score_Z=None, grad=None, cp_upper=None,
                  tile_bound=None, stream=None):
    _check("cse_calibrate", _L.cse_calibrate(h, seed, alpha, _ptr(alpha_prime), _ptr(k), _ptr(lambda_tile),
                                             _ptr(lambda_global), _ptr(reject_at_lambda), delta,
                                             _ptr(reject), _ptr(score_T), _ptr(score_Z), _ptr(grad),
                                             _ptr(cp_upper), _ptr(tile_bound), _stream(stream)))


def cse_calibrate_noalloc(h, seed, alpha, alpha_prime, k, lambda_tile, lambda_global, reject_at_lambda=None,
                          delta=0.01, reject=None, score_T=None, score_Z=None, grad=None, cp_upper=None,
                          tile_bound=None, stream=None):
    _check("cse_calibrate_noalloc", _L.cse_calibrate_noalloc(
        h, seed, alpha, _ptr(alpha_prime), _ptr(k), _ptr(lambda_tile), _ptr(lambda_global), _ptr(reject_at_lambda),
        delta, _ptr(reject), _ptr(score_T), _ptr(score_Z), _ptr(grad), _ptr(cp_upper), _ptr(tile_bound),
        _stream(stream)))


# bytes of the static calibration workspace of cse_calibrate_noalloc (CSE_NOALLOC_SCRATCH_BYTES)
NOALLOC_SCRATCH_BYTES = 64 << 20


def cse_bound(h, mode, R, a, level, out, q_star=None, stream=None):
    _check("cse_bound", _L.cse_bound(h, mode, _ptr(R), _ptr(a), level, _ptr(out), _ptr(q_star),
                                     _stream(stream)))


def cse_simulate_per_tile(h, seed, tile_begin, tile_end, reject, stream=None):
    _check("cse_simulate_per_tile", _L.cse_simulate_per_tile(h, seed, tile_begin, tile_end, _ptr(reject),
                                                             _stream(stream)))


def cse_plan_validate(h, seed, delta, reject, score_T, score_Z, grad, cp_upper, tile_bound, q_star=None):
    out = ctypes.c_void_p()
    _check("cse_plan_validate", _L.cse_plan_validate(h, seed, delta, _ptr(reject), _ptr(score_T), _ptr(score_Z),
                                                     _ptr(grad), _ptr(cp_upper), _ptr(tile_bound), _ptr(q_star),
                                                     ctypes.byref(out)))
    return out


def cse_plan_calibrate(h, seed, alpha, alpha_prime, k, lambda_tile, lambda_global, reject_at_lambda=None,
                       delta=0.01, reject=None, score_T=None, score_Z=None, grad=None, cp_upper=None,
                       tile_bound=None):
    out = ctypes.c_void_p()
    _check("cse_plan_calibrate", _L.cse_plan_calibrate(
        h, seed, alpha, _ptr(alpha_prime), _ptr(k), _ptr(lambda_tile), _ptr(lambda_global), _ptr(reject_at_lambda),
        delta, _ptr(reject), _ptr(score_T), _ptr(score_Z), _ptr(grad), _ptr(cp_upper), _ptr(tile_bound),
        ctypes.byref(out)))
    return out


def cse_plan_launch(plan, stream=None):
    _check("cse_plan_launch", _L.cse_plan_launch(plan, _stream(stream)))


def cse_plan_nodes(plan) -> int:
    return int(_L.cse_plan_nodes(plan))


def cse_plan_destroy(plan):
    _check("cse_plan_destroy", _L.cse_plan_destroy(plan))


def cse_taylor(h, f, grad, bound, vertex=None, point=None, stream=None):
    _check("cse_taylor", _L.cse_taylor(h, _ptr(f), _ptr(grad), _ptr(bound), _ptr(vertex), _ptr(point),
                                       _stream(stream)))


def cse_validate_lower(h, R, delta, cp_lower, lower, q_star=None, stream=None):
    _check("cse_validate_lower", _L.cse_validate_lower(h, _ptr(R), delta, _ptr(cp_lower), _ptr(lower), _ptr(q_star),
                                                       _stream(stream)))


def cse_confidence_set(h, s_obs, s_stride, lambda_tile, coef, link, keep, e_lo, e_hi, e_range, stream=None):
    c = np.ascontiguousarray(coef, np.float64)
    _check("cse_confidence_set", _L.cse_confidence_set(h, _ptr(s_obs), s_stride, _ptr(lambda_tile), _ptr(c), link,
                                                       _ptr(keep), _ptr(e_lo), _ptr(e_hi), _ptr(e_range),
                                                       _stream(stream)))


def cse_calibrate_tiebreak(h, seed, alpha, alpha_prime, k, lambda_tile, u_tile, lambda_global, u_global,
                           reject_at_lambda, stream=None):
    _check("cse_calibrate_tiebreak", _L.cse_calibrate_tiebreak(
        h, seed, alpha, _ptr(alpha_prime), _ptr(k), _ptr(lambda_tile), _ptr(u_tile), _ptr(lambda_global),
        _ptr(u_global), _ptr(reject_at_lambda), _stream(stream)))


def cse_adagrid_decide(rule, radii, sims, tile_box, a, b, c):
    """Host call: per-box decision codes (0 done, 1 split, 2 double N, 3 stuck)."""
    radii = np.ascontiguousarray(radii, np.float64)
    sims = np.ascontiguousarray(sims, np.int32)
    tb = np.ascontiguousarray(tile_box, np.int64)
    a, b, c = (np.ascontiguousarray(x, np.float64) for x in (a, b, c))
    dec = np.zeros(len(sims), np.int32)
    _check("cse_adagrid_decide", _L.cse_adagrid_decide(ctypes.byref(rule), len(sims), _ptr(radii), _ptr(sims),
                                                       len(tb), _ptr(tb), _ptr(a), _ptr(b), _ptr(c), _ptr(dec)))
    return dec


def cse_adagrid_apply(theta, radii, sims, decision):
    """Host call: the next box list (theta, radii, sims, parent, changed)."""
    theta = np.ascontiguousarray(theta, np.float64)
    radii = np.ascontiguousarray(radii, np.float64)
    sims = np.ascontiguousarray(sims, np.int32)
    dec = np.ascontiguousarray(decision, np.int32)
    d = theta.shape[1]
    n = ctypes.c_int64()
    _check("cse_adagrid_apply", _L.cse_adagrid_apply(d, len(sims), _ptr(theta), _ptr(radii), _ptr(sims), _ptr(dec),
                                                     0, None, None, None, None, None, ctypes.byref(n)))
    m = n.value
    th, rd = np.zeros((m, d)), np.zeros((m, d))
    sm, par, ch = np.zeros(m, np.int32), np.zeros(m, np.int64), np.zeros(m, np.int32)
    _check("cse_adagrid_apply", _L.cse_adagrid_apply(d, len(sims), _ptr(theta), _ptr(radii), _ptr(sims), _ptr(dec),
                                                     m, _ptr(th), _ptr(rd), _ptr(sm), _ptr(par), _ptr(ch),
                                                     ctypes.byref(n)))
    return th, rd, sm, par, ch.astype(bool)


def cse_autotune(h, seed=0, max_trials=1 << 24, stream=None):
    """Pick the fused kernel's launch shape on this device; returns (value, grid)."""
    out = np.zeros(2, np.int64)
    _check("cse_autotune", _L.cse_autotune(h, seed, max_trials, _ptr(out), _stream(stream)))
    return int(out[0]), int(out[1])


CSE_OPT_B2_MARGIN = 1   # 2-arm calibration: bracket margin (standard deviations of the count)
CSE_OPT_H4_MARGIN = 2   # 4-arm calibration: bracket margin (standard deviations of the pilot rank)
CSE_OPT_H4_BRACKET = 3   # 4-arm calibration: 1 = bracketed keys, 0 = every float32 key in HBM (default)


def cse_platten_set_option(h, option, value):
    """Set a platten tuning option (CSE_OPT_B2_MARGIN, CSE_OPT_H4_BRACKET, CSE_OPT_H4_MARGIN)."""
    _check("cse_platten_set_option", _L.cse_platten_set_option(h, int(option), float(value)))


def cse_work_counters(h, stream=None) -> dict:
    """Phase II/III design: trials, posterior looks (Phase II, Phase III) and Newton steps of
    the last simulation launch.  2-arm design: `trials` holds the tiles the last calibration
    left to the exact full-histogram pass; 4-arm design: the tiles whose k-th key the last
    bracketed calibration selected from regenerated keys."""
    out = np.zeros(4, np.int64)
    _check("cse_work_counters", _L.cse_work_counters(h, _ptr(out), _stream(stream)))
    return dict(trials=int(out[0]), looks_phase2=int(out[1]), looks_phase3=int(out[2]),
                newton_steps=int(out[3]))


def cse_platten_stats(h) -> dict:
    out = np.zeros(12, np.int64)
    _check("cse_platten_stats", _L.cse_platten_stats(h, _ptr(out)))
    keys = ("n_tiles", "n_batches", "n_work_items", "n_key_slots", "total_sims", "tiles_per_batch",
            "max_sims", "batch_sims", "group_sims", "n_sim_classes", "table_build_us", "launch_shape")
    return {k: int(v) for k, v in zip(keys, out)}


def cse_posterior_table(h, stream=None) -> torch.Tensor:
    """The 4-arm design's table [(n+1)^4, 4] float32 (1 - P_1, 1 - P_2, 1 - P_3, 0) on the device."""
    n = ctypes.c_int64()
    _check("cse_posterior_table", _L.cse_posterior_table(h, None, 0, ctypes.byref(n), None))
    out = torch.empty((n.value, 4), dtype=torch.float32, device="cuda")
    _check("cse_posterior_table", _L.cse_posterior_table(h, _ptr(out), out.numel(), ctypes.byref(n),
                                                         _stream(stream)))
    return out


def cse_profile_enable(on: bool = True):
    _check("cse_profile_enable", _L.cse_profile_enable(1 if on else 0))


def cse_profile_get(name: str):
    n = ctypes.c_int64()
    ms = ctypes.c_double()
    _check("cse_profile_get", _L.cse_profile_get(name.encode(), ctypes.byref(n), ctypes.byref(ms)))
    return int(n.value), float(ms.value)


def cse_profile_reset():
    _check("cse_profile_reset", _L.cse_profile_reset())


# ------------------------------------------------------------------ convenience layer
@dataclass
class Platten:
    """A platten on the current device: the handle plus its tile description."""
    handle: ctypes.c_void_p
    design: cse_design
    n_tiles: int
    d: int
    tiles: dict

    @classmethod
    def create(cls, kind, theta, radii, sims, cut=None, keep_all=False, theta0=None):
        des = make_design(kind, cut, theta0=theta0)
        h = cse_platten_create(des, theta, radii, sims, CSE_PLATTEN_KEEP_ALL if keep_all else 0)
        n = cse_platten_size(h)
        tiles = cse_platten_describe(h)
        tiles["theta"], tiles["radii"] = cse_platten_tiles(h, n, des.n_arms)
        return cls(h, des, n, des.n_arms, tiles)

    def close(self):
        if self.handle:
            cse_platten_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _alloc(self, device):
        n, d = self.n_tiles, self.d
        dev = torch.device(device)
        kind = self.design.kind
        return dict(
            reject=torch.empty(n, dtype=torch.int32, device=dev),
            score_T=(torch.empty((n, 2 * d), dtype=torch.int64, device=dev) if kind == CSE_PHASE23 else
                     torch.empty((n, d), dtype=torch.int64, device=dev) if kind != CSE_ZTEST1 else None),
            score_Z=torch.empty(n, dtype=torch.float64, device=dev) if kind == CSE_ZTEST1 else None,
            grad=torch.empty((n, d), dtype=torch.float64, device=dev),
        )

    def simulate(self, seed=0, device="cuda"):
        o = self._alloc(device)
        cse_simulate(self.handle, seed, o["reject"], o["score_T"], o["score_Z"], o["grad"])
        return o

    def validate(self, seed=0, delta=0.01, device="cuda"):
        o = self._alloc(device)
        n = self.n_tiles
        o["cp_upper"] = torch.empty(n, dtype=torch.float64, device=device)
        o["tile_bound"] = torch.empty(n, dtype=torch.float64, device=device)
        o["q_star"] = torch.empty(n, dtype=torch.float64, device=device)
        cse_validate(self.handle, seed, delta, o["reject"], o["score_T"], o["score_Z"], o["grad"],
                     o["cp_upper"], o["tile_bound"], o["q_star"])
        return o

    def calibrate(self, seed=0, alpha=0.025, delta=0.01, with_validation=True, device="cuda", noalloc=False):
        n = self.n_tiles
        o = self._alloc(device) if with_validation else {}
        o.update(alpha_prime=torch.empty(n, dtype=torch.float64, device=device),
                 k=torch.empty(n, dtype=torch.int32, device=device),
                 lambda_tile=torch.empty(n, dtype=torch.float64, device=device),
                 lambda_global=torch.empty(1, dtype=torch.float64, device=device),
                 reject_at_lambda=torch.empty(n, dtype=torch.int32, device=device))
        if with_validation:
            o["cp_upper"] = torch.empty(n, dtype=torch.float64, device=device)
            o["tile_bound"] = torch.empty(n, dtype=torch.float64, device=device)
        fn = cse_calibrate_noalloc if noalloc else cse_calibrate
        fn(self.handle, seed, alpha, o["alpha_prime"], o["k"], o["lambda_tile"], o["lambda_global"],
           o["reject_at_lambda"], delta, o.get("reject"), o.get("score_T"), o.get("score_Z"),
           o.get("grad"), o.get("cp_upper"), o.get("tile_bound"))
        return o

    def taylor(self, f, grad, device="cuda"):
        """Taylor comparison bound over each tile and its worst-case candidate vertex (Section 4.3)."""
        n = self.n_tiles
        out = dict(bound=torch.empty(n, dtype=torch.float64, device=device),
                   vertex=torch.empty(n, dtype=torch.int32, device=device),
                   point=torch.empty((n, self.d), dtype=torch.float64, device=device))
        cse_taylor(self.handle, f, grad, out["bound"], out["vertex"], out["point"])
        return out

    def validate_lower(self, R, delta=0.01, device="cuda"):
        """Lower side of the two-sided band (Remark 2) from rejection counts R (device int32)."""
        n = self.n_tiles
        out = dict(cp_lower=torch.empty(n, dtype=torch.float64, device=device),
                   lower=torch.empty(n, dtype=torch.float64, device=device),
                   q_star=torch.empty(n, dtype=torch.float64, device=device))
        cse_validate_lower(self.handle, R, delta, out["cp_lower"], out["lower"], out["q_star"])
        return out

    def confidence_set(self, s_obs, lambda_tile, coef, link="linear", device="cuda"):
        """Confidence set from a calibration (Section 8): keep mask, per-tile range of e and the
        range over kept tiles.  s_obs: a float or a per-tile float64 tensor."""
        n = self.n_tiles
        if isinstance(s_obs, torch.Tensor):
            s, stride = s_obs.to(device=device, dtype=torch.float64).contiguous(), 1
        else:
            s, stride = torch.full((1,), float(s_obs), dtype=torch.float64, device=device), 0
        out = dict(keep=torch.empty(n, dtype=torch.int32, device=device),
                   e_lo=torch.empty(n, dtype=torch.float64, device=device),
                   e_hi=torch.empty(n, dtype=torch.float64, device=device),
                   e_range=torch.empty(2, dtype=torch.float64, device=device))
        cse_confidence_set(self.handle, s, stride, lambda_tile, coef, {"linear": 0, "expit": 1}[link],
                           out["keep"], out["e_lo"], out["e_hi"], out["e_range"])
        return out

    def calibrate_tiebreak(self, seed=0, alpha=0.025, device="cuda"):
        """Randomised calibration: thresholds (lambda_i, c_i) on the pair (S, u).  The uint32
        values c are returned in int32 tensors (reinterpret with .view(numpy.uint32))."""
        n = self.n_tiles
        o = dict(alpha_prime=torch.empty(n, dtype=torch.float64, device=device),
                 k=torch.empty(n, dtype=torch.int32, device=device),
                 lambda_tile=torch.empty(n, dtype=torch.float64, device=device),
                 u_tile=torch.empty(n, dtype=torch.int32, device=device),
                 lambda_global=torch.empty(1, dtype=torch.float64, device=device),
                 u_global=torch.empty(1, dtype=torch.int32, device=device),
                 reject_at_lambda=torch.empty(n, dtype=torch.int32, device=device))
        cse_calibrate_tiebreak(self.handle, seed, alpha, o["alpha_prime"], o["k"], o["lambda_tile"], o["u_tile"],
                               o["lambda_global"], o["u_global"], o["reject_at_lambda"])
        return o

    def bound(self, mode, R=None, a=None, level=0.01, device="cuda"):
        out = torch.empty(self.n_tiles, dtype=torch.float64, device=device)
        q = torch.empty(self.n_tiles, dtype=torch.float64, device=device)
        cse_bound(self.handle, mode, R, a, level, out, q)
        return out, q


class TIE(torch.autograd.Function):
    """Type I Error of each box (rejection rate of the design's fixed rule) with its
    score-function gradient, both from one simulation pass.

    forward(theta [n_boxes, d] float64, radii, sims, kind, seed) -> R / N per box;
    backward returns grad_out * (sum_rej T(x) - R grad A(theta)) / N.  Single-hypothesis
    designs only (each box is one tile)."""

    @staticmethod
    def forward(ctx, theta, radii, sims, kind, seed):
        th = theta.detach().to("cpu", torch.float64).numpy()
        P = Platten.create(kind, th, np.asarray(radii, np.float64), np.asarray(sims, np.int32), keep_all=True)
        try:
            if P.n_tiles != th.shape[0]:
                raise ValueError("TIE needs one tile per box (single-hypothesis design)")
            o = P.simulate(seed, device=theta.device if theta.is_cuda else "cuda")
            N = torch.as_tensor(np.asarray(sims, np.float64), device=o["reject"].device)
            f = o["reject"].to(torch.float64) / N
            g = o["grad"]
            torch.cuda.current_stream().synchronize()
        finally:
            P.close()
        ctx.save_for_backward(g.to(theta.device))
        return f.to(theta.device)

    @staticmethod
    def backward(ctx, gout):
        (g,) = ctx.saved_tensors
        return gout[:, None] * g, None, None, None, None
