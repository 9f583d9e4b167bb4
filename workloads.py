"""Seeded synthetic workloads (tile grids) shared by the tests, the benchmark and smoke().

This module holds *inputs only*: tile centres, half-widths and simulations per
tile, laid out the way the case studies of the paper lay out their grids
(equally spaced centres of equal boxes, Section 6.4 and Section 10.2; n = 35
patients per arm, Section 10.1; alpha = 2.5%, Section 1; 2,048 or more
simulations per tile, Section 10.2).  It contains none of the method's
arithmetic: no thresholds, no null-hypothesis clipping, no vertices, no
statistics.  Each side (the oracle and the HIP library) derives those itself.

Every grid is returned as a dict with
    theta : float64 [n_tiles, d]   tile centres (natural parameters: logits or means)
    radii : float64 [n_tiles, d]   tile half-widths
    sims  : int32   [n_tiles]      simulations per tile
plus the scalars that go with the workload (seed, delta, alpha).
"""
from __future__ import annotations

import numpy as np

N_PER_ARM = 35


def _centres(lo: float, hi: float, m: int) -> np.ndarray:
    """m equally spaced box centres covering [lo, hi] with equal boxes."""
    w = (hi - lo) / m
    return lo + (np.arange(m, dtype=np.float64) + 0.5) * w


def ztest_1d(n_tiles: int = 64, sims: int = 10_000, lo: float = -1.0, hi: float = 0.0,
             seed: int = 0) -> dict:
    """1-D normal z-test grid: equal tiles over [lo, hi] (Section 6.4, Section 7.4)."""
    c = _centres(lo, hi, n_tiles)
    r = (hi - lo) / (2 * n_tiles)
    return dict(name=f"ztest1d_{n_tiles}x{sims}", design="ztest1",
                theta=c[:, None].copy(), radii=np.full((n_tiles, 1), r),
                sims=np.full(n_tiles, sims, np.int32), seed=seed,
                delta=0.01, alpha=0.025)


def binom2_grid(m: int = 256, sims: int = 8192, lo: float = -3.0, hi: float = 1.0,
                lower_triangle: bool = True, seed: int = 0) -> dict:
    """2-arm binomial grid over (theta0, theta1) in [lo, hi]^2, m x m boxes.

    With lower_triangle, keeps the boxes whose theta1 index is <= the theta0
    index (the boxes that touch theta1 <= theta0), in row-major order of
    (theta0 index, theta1 index).
    """
    c = _centres(lo, hi, m)
    r = (hi - lo) / (2 * m)
    i0, i1 = np.meshgrid(np.arange(m), np.arange(m), indexing="ij")
    i0 = i0.ravel(); i1 = i1.ravel()
    if lower_triangle:
        keep = i1 <= i0
        i0 = i0[keep]; i1 = i1[keep]
    theta = np.stack([c[i0], c[i1]], axis=1)
    n = theta.shape[0]
    return dict(name=f"binom2_{m}x{m}{'_tri' if lower_triangle else ''}x{sims}",
                design="binom2", theta=theta, radii=np.full((n, 2), r),
                sims=np.full(n, sims, np.int32), seed=seed, delta=0.01, alpha=0.025)


def hier4_grid(m: int = 16, sims: int = 32_768, lo: float = -1.0, hi: float = 1.0,
               seed: int = 0) -> dict:
    """4-arm grid, m^4 equal boxes on [lo, hi]^4, arm 0 first (row-major)."""
    c = _centres(lo, hi, m)
    r = (hi - lo) / (2 * m)
    g = np.stack(np.meshgrid(c, c, c, c, indexing="ij"), axis=-1).reshape(-1, 4)
    n = g.shape[0]
    return dict(name=f"hier4_{m}^4x{sims}", design="hier4", theta=g.copy(),
                radii=np.full((n, 4), r), sims=np.full(n, sims, np.int32), seed=seed,
                delta=0.01, alpha=0.025)


def phase23_grid(shape=(4, 4, 4, 4), sims=None, lo: float = -0.9946, hi: float = 1.1527,
                 seed: int = 0, sims_seed: int = 0, lam: float = 0.06253) -> dict:
    """4-arm grid for the Phase II/III design: shape[a] equal boxes per arm on [lo, hi] (the
    logit box of p in [27%, 76%], Section 10.2), arm 0 first (row-major).  sims: an int for
    equal counts, or None for the uneven 2^(11+g), g uniform on {0..5} (PCG64(sims_seed))."""
    cs = [_centres(lo, hi, m) for m in shape]
    rs = [(hi - lo) / (2 * m) for m in shape]
    g = np.stack(np.meshgrid(*cs, indexing="ij"), axis=-1).reshape(-1, 4)
    n = g.shape[0]
    radii = np.tile(np.array(rs), (n, 1))
    sm = np.full(n, sims, np.int32) if sims is not None else uneven_sims(n, sims_seed)
    tag = "x".join(str(m) for m in shape)
    return dict(name=f"phase23_{tag}x{'uneven' if sims is None else sims}", design="phase23",
                theta=g.copy(), radii=radii, sims=sm, seed=seed, delta=0.01, alpha=0.025, cut=lam)


def basket_grid(m: int = 16, sims: int = 32_768, lo: float = -3.5, hi: float = 1.0, seed: int = 0) -> dict:
    """Basket design grid, m^4 equal boxes on [lo, hi]^4 (Section 10.1's theta range [-3.5, 1]^4),
    row-major; the design cuts the boxes that straddle theta_a = logit(0.15) into pieces."""
    c = _centres(lo, hi, m)
    r = (hi - lo) / (2 * m)
    g = np.stack(np.meshgrid(c, c, c, c, indexing="ij"), axis=-1).reshape(-1, 4)
    n = g.shape[0]
    return dict(name=f"basket4_{m}^4x{sims}", design="basket4", theta=g.copy(), radii=np.full((n, 4), r),
                sims=np.full(n, sims, np.int32), seed=seed, delta=0.01, alpha=0.025, cut=0.15)


def uneven_sims(n_tiles: int, seed: int = 0, lo_pow: int = 11, n_classes: int = 6) -> np.ndarray:
    """Simulations per tile 2^(lo_pow+g), g uniform on {0..n_classes-1} (PCG64 seeded)."""
    g = np.random.Generator(np.random.PCG64(seed)).integers(0, n_classes, n_tiles)
    return (2 ** (lo_pow + g)).astype(np.int32)


def subsample(w: dict, idx) -> dict:
    """The same workload restricted to the tiles `idx` (order kept)."""
    idx = np.asarray(idx)
    out = dict(w)
    out["theta"] = w["theta"][idx].copy()
    out["radii"] = w["radii"][idx].copy()
    out["sims"] = w["sims"][idx].copy()
    out["name"] = w["name"] + f"_sub{len(idx)}"
    return out


# The benchmark workloads, by what they are.
def ztest1d_64() -> dict:
    """64 tiles on [-1, 0], half-width 1/128, 10,000 sims, seed 0."""
    return ztest_1d(64, 10_000)


def binom2_256_tri() -> dict:
    """2-arm n=35 binomial, 256x256 boxes on [-3,1]^2 kept to theta1<=theta0, 8,192 sims."""
    return binom2_grid(256, 8192)


def binom2_1024_full() -> dict:
    """2-arm n=35 binomial, all 1024x1024 boxes on [-3,1]^2, 16,384 sims."""
    return binom2_grid(1024, 16_384, lower_triangle=False)


def hier4_16() -> dict:
    """4-arm n=35 hierarchical design, 16^4 boxes on [-1,1]^4, 32,768 sims."""
    return hier4_grid(16, 32_768)


def basket4_16() -> dict:
    """Basket design, 16^4 boxes on [-3.5, 1]^4, 32,768 sims per piece."""
    return basket_grid(16, 32_768)


def phase23_c5() -> dict:
    """Phase II/III design, 16 x 16 x 32 x 32 boxes (2^18) on the logit box [-0.9946, 1.1527]^4,
    2^(11+g) sims per box with g uniform on {0..5} (PCG64(0)), seed 0, lambda 0.06253."""
    return phase23_grid((16, 16, 32, 32), None)
