"""Seeded synthetic MDS problems shaped like the paper's workloads.

This module only draws inputs; it holds none of the likelihood arithmetic.
Distances of the *true* configuration come from ``scipy.spatial.distance.cdist``
and the truncated-normal draws from ``scipy.special.ndtr``/``ndtri`` (the
inverse-CDF method), so both the oracle side and the GPU side can be fed from
it without sharing any code of the method.

Recipe (one problem):
  * X_true ~ N(0, I_D) * 3, from ``seed``.
  * Optional duplicates: a fraction of points becomes a copy of another point
    plus ``dup_jitter * N(0, I_D)`` (stream ``seed + 4``).
  * y_ij for i > j ~ N(delta_ij, sigma^2) truncated to (0, inf), with
    delta_ij = ||x_i - x_j|| of X_true (the observation model of Section 2.1,
    Eq. 1), drawn by inverse CDF: y = delta + sigma * Phi^{-1}(Phi(-delta/sigma)
    + u * Phi(delta/sigma)), u ~ U(0,1) from stream ``seed + 1`` in row-major
    order of the packed lower triangle.  Y is mirrored and has a zero diagonal.
  * Optional missing mask: symmetric Bernoulli(rate) over i > j, stream
    ``seed + 2``, mirrored, zero diagonal.
  * Evaluation point X = X_true + N(0, 0.1^2) (stream ``seed + 3``), with the
    duplicate points re-copied from their sources plus fresh jitter so that
    they stay near-coincident where the likelihood is evaluated.
"""
from __future__ import annotations

import concurrent.futures as cf
from dataclasses import dataclass, field

import numpy as np
from scipy.spatial.distance import cdist
from scipy.special import ndtr, ndtri

_ROW_BLOCK = 1024


@dataclass
class Problem:
    n: int
    d: int
    sigma: float
    x_true: np.ndarray            # N x D float64
    x: np.ndarray                 # N x D float64, evaluation point
    y: np.ndarray                 # N x N float64, symmetric, zero diagonal
    mask: np.ndarray | None       # N x N uint8 (1 = missing) or None
    seed: int
    recipe: dict = field(default_factory=dict)


def _duplicates(n, d, frac, rng):
    k = int(round(frac * n))
    if k <= 0:
        return np.zeros(0, np.int64), np.zeros(0, np.int64)
    targets = rng.choice(n, size=k, replace=False)
    others = np.setdiff1d(np.arange(n), targets)
    sources = others[rng.integers(0, others.size, size=k)]
    return targets.astype(np.int64), sources.astype(np.int64)


def _mirror_lower(a):
    """Copy the strict lower triangle of a square array onto its upper one."""
    n = a.shape[0]
    b = _ROW_BLOCK
    for i0 in range(0, n, b):
        i1 = min(n, i0 + b)
        blk = a[i0:i1, i0:i1]
        lower = np.tril(blk, -1)
        a[i0:i1, i0:i1] = lower + lower.T + np.diag(np.diag(blk))
        for j0 in range(0, i0, b):
            j1 = min(n, j0 + b)
            a[j0:j1, i0:i1] = a[i0:i1, j0:j1].T


def _tn_block(delta, u, sigma):
    lo = ndtr(-delta / sigma)           # P(y <= 0) under N(delta, sigma^2), <= 1/2
    z = ndtri(np.clip(lo + u * (1.0 - lo), 1e-300, 1.0 - 2.0 ** -53))
    return np.maximum(delta + sigma * z, np.finfo(np.float64).tiny)


def truncated_normal_y(x_true, sigma, rng, threads: int = 8):
    """Symmetric Y with y_ij ~ N(delta_ij, sigma^2) I(y_ij > 0) for i > j.
    The uniforms are consumed row by row over j < i (row-major order of the
    packed lower triangle), whatever the block size used to draw them; the
    inverse-CDF transform of each block then runs on a thread pool."""
    n = x_true.shape[0]
    y = np.zeros((n, n), dtype=np.float64)

    def work(i0, i1, u):
        dist = cdist(x_true[i0:i1], x_true[:i1])
        lower = np.arange(i1)[None, :] < np.arange(i0, i1)[:, None]
        blk = np.zeros((i1 - i0, i1), dtype=np.float64)
        blk[lower] = _tn_block(dist[lower], u, sigma)
        y[i0:i1, :i1] = blk

    with cf.ThreadPoolExecutor(max(1, threads)) as ex:
        futs = []
        for i0 in range(1, n, _ROW_BLOCK):
            i1 = min(n, i0 + _ROW_BLOCK)
            cnt = (i1 - i0) * (i0 + i1 - 1) // 2        # sum of i over the block's rows
            futs.append(ex.submit(work, i0, i1, rng.random(cnt)))
        for f in futs:
            f.result()
    _mirror_lower(y)
    np.fill_diagonal(y, 0.0)
    return y


def symmetric_mask(n, rate, rng):
    if rate <= 0.0:
        return None
    m = np.zeros((n, n), dtype=np.uint8)
    for i0 in range(1, n, _ROW_BLOCK):
        i1 = min(n, i0 + _ROW_BLOCK)
        lower = np.arange(i1)[None, :] < np.arange(i0, i1)[:, None]
        blk = np.zeros((i1 - i0, i1), dtype=np.uint8)
        blk[lower] = rng.random(int(lower.sum())) < rate
        m[i0:i1, :i1] = blk
    _mirror_lower(m)
    np.fill_diagonal(m, 0)
    return m


def make_problem(n: int, d: int, sigma: float, *, seed: int = 0, missing: float = 0.0,
                 dup_frac: float = 0.0, dup_jitter: float = 1e-4,
                 eval_noise: float = 0.1) -> Problem:
    rng_x = np.random.Generator(np.random.PCG64(seed))
    x_true = rng_x.standard_normal((n, d)) * 3.0
    rng_dup = np.random.Generator(np.random.PCG64(seed + 4))
    targets, sources = _duplicates(n, d, dup_frac, rng_dup)
    if targets.size:
        x_true[targets] = x_true[sources] + dup_jitter * rng_dup.standard_normal((targets.size, d))
    y = truncated_normal_y(x_true, sigma, np.random.Generator(np.random.PCG64(seed + 1)))
    mask = symmetric_mask(n, missing, np.random.Generator(np.random.PCG64(seed + 2)))
    rng_e = np.random.Generator(np.random.PCG64(seed + 3))
    x = x_true + eval_noise * rng_e.standard_normal((n, d))
    if targets.size:
        x[targets] = x[sources] + dup_jitter * rng_dup.standard_normal((targets.size, d))
    recipe = dict(n=n, d=d, sigma=sigma, seed=seed, missing=missing, dup_frac=dup_frac,
                  dup_jitter=dup_jitter, eval_noise=eval_noise, x_scale=3.0)
    return Problem(n, d, float(sigma), x_true, x, y, mask, seed, recipe)


def device_problem(n: int, d: int, sigma: float, *, seed: int = 0, dtype=None,
                   device="cuda", eval_noise: float = 0.1, block_rows: int = 1024,
                   missing: float = 0.0):
    """A problem of the same recipe (no missing pairs, no duplicates) whose
    symmetric Y is drawn directly in device memory, for sizes where the host
    recipe would take minutes (N = 10^5: 10^10 entries, 80 GB in FP64).

    X_true and the evaluation point come from the same PCG64 streams as
    ``make_problem``; the truncated-normal draws use the same inverse-CDF
    transform in FP64 (torch's ndtr/ndtri) with uniforms from torch's device
    generator seeded with ``seed + 1`` (one (rows x columns) draw per block of
    ``block_rows`` rows, lower triangle used), so Y follows the same
    distribution as the host recipe but not the same values.  ``missing``
    marks that fraction of the pairs missing (a symmetric Bernoulli draw from
    a device generator seeded with ``seed + 2``) by setting them to NaN, which
    the library reads as missing.  Returns (x_true, x) as host arrays and Y as
    an N x N device tensor of ``dtype`` (float64 by default).
    """
    import torch

    dtype = torch.float64 if dtype is None else dtype
    rng_x = np.random.Generator(np.random.PCG64(seed))
    x_true = rng_x.standard_normal((n, d)) * 3.0
    rng_e = np.random.Generator(np.random.PCG64(seed + 3))
    x = x_true + eval_noise * rng_e.standard_normal((n, d))
    xt = torch.as_tensor(x_true, device=device)
    y = torch.empty((n, n), dtype=dtype, device=device)
    gen = torch.Generator(device=device)
    gen.manual_seed(seed + 1)
    hi = 1.0 - 2.0 ** -53
    for i0 in range(0, n, block_rows):
        i1 = min(n, i0 + block_rows)
        delta = torch.zeros((i1 - i0, i1), dtype=torch.float64, device=device)
        for k in range(d):
            delta += (xt[i0:i1, k, None] - xt[None, :i1, k]).square_()
        delta.sqrt_()
        u = torch.rand((i1 - i0, i1), generator=gen, dtype=torch.float64, device=device)
        lo = torch.special.ndtr(-delta / sigma)
        z = torch.special.ndtri((lo + u * (1.0 - lo)).clamp_(1e-300, hi))
        y[i0:i1, :i1] = (delta + sigma * z).clamp_(min=np.finfo(np.float64).tiny)
        del delta, u, lo, z
    if missing > 0.0:
        gm = torch.Generator(device=device)
        gm.manual_seed(seed + 2)
        for i0 in range(0, n, block_rows):
            i1 = min(n, i0 + block_rows)
            drop = torch.rand((i1 - i0, i1), generator=gm, device=device) < missing
            y[i0:i1, :i1].masked_fill_(drop, float("nan"))
    # mirror the strict lower triangle, zero diagonal
    for i0 in range(0, n, block_rows):
        i1 = min(n, i0 + block_rows)
        blk = torch.tril(y[i0:i1, i0:i1], -1)
        y[i0:i1, i0:i1] = blk + blk.T
        if i0 > 0:
            y[:i0, i0:i1] = y[i0:i1, :i0].T
    return x_true, x, y


# Workload presets: sizes, sigma, missing rate and duplicates of the paper's
# application scale (N = 5392 locations, Section 3) and of the precision,
# differentiation and batched forms built around it.
PRESETS = {
    "small_fp64": dict(n=1000, d=2, sigma=0.5, seed=1000),
    "paper_fp64": dict(n=5392, d=2, sigma=0.3, missing=0.15, seed=5392),
    "paper_fp32_d2": dict(n=5392, d=2, sigma=0.5, dup_frac=0.01, seed=5393),
    "paper_fp32_d6_tight": dict(n=5392, d=6, sigma=0.05, dup_frac=0.01, seed=5394),
    "large_fp32_d2": dict(n=20000, d=2, sigma=0.5, dup_frac=0.01, seed=20000),
    "large_fp32_d6_tight": dict(n=20000, d=6, sigma=0.05, dup_frac=0.01, seed=20001),
    "paper_fp32_d2_tight": dict(n=5392, d=2, sigma=0.05, dup_frac=0.01, seed=5395),
    "paper_fp32_d6": dict(n=5392, d=6, sigma=0.5, dup_frac=0.01, seed=5396),
    "large_fp32_d2_tight": dict(n=20000, d=2, sigma=0.05, dup_frac=0.01, seed=20002),
    "large_fp32_d6": dict(n=20000, d=6, sigma=0.5, dup_frac=0.01, seed=20003),
}

# The precision form's grid: N in {5392, 20000} x D in {2, 6} x sigma in
# {0.5, 0.05}, FP32 Y, 1% of the points near-duplicates (jitter 1e-4).
PRECISION_PRESETS = ("paper_fp32_d2", "paper_fp32_d2_tight", "paper_fp32_d6",
                     "paper_fp32_d6_tight", "large_fp32_d2", "large_fp32_d2_tight",
                     "large_fp32_d6", "large_fp32_d6_tight")


def preset(name: str, **override) -> Problem:
    kw = dict(PRESETS[name])
    kw.update(override)
    return make_problem(**kw)


def batch_specs(count: int = 64, seed: int = 64, n_lo: int = 500, n_hi: int = 8000,
                dims=(2, 4, 6), missing: float = 0.10):
    """Per-problem (n, d, sigma, seed) for the batched form: N ~ U[n_lo, n_hi],
    D uniform over ``dims``, sigma ~ U(0.2, 1.0), 10% missing."""
    rng = np.random.Generator(np.random.PCG64(seed))
    specs = []
    for k in range(count):
        n = int(rng.integers(n_lo, n_hi + 1))
        d = int(rng.choice(np.asarray(dims)))
        s = float(rng.uniform(0.2, 1.0))
        specs.append(dict(n=n, d=d, sigma=s, missing=missing, seed=seed * 1000 + 10 * k))
    return specs
