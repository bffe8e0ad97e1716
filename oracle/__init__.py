"""Plain serial FP64 CPU oracle for the truncated-normal MDS likelihood path.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU-baseline
leg of the bench may import this package; the product library never does.
The arithmetic lives in ``mds_oracle.c`` (compiled with gcc -O2, no fast-math);
this module only marshals numpy arrays into it.

Functions follow Holbrook et al., "Massive parallelization boosts big
Bayesian multidimensional scaling":
  * ``log_phi``/``mills``   -- ln Phi(t) and phi(t)/Phi(t) (Eq. 2, Eq. 9)
  * ``evaluate``            -- L, dL/dX, dL/dsigma (Eq. 2, Eq. 9); with
                               ``truncated=False`` the model without the
                               truncation to y > 0 (the scaling appendix)
  * ``grad_rows``/``grad_rows_given`` -- listed gradient rows of Eq. (9)
  * ``leapfrog``            -- one HMC leapfrog trajectory (Section 2.3)
  * ``philox4x32_10``, ``uniform_open``, ``momentum``, ``accept_uniform``,
    ``hmc_step``            -- the random draws and one HMC transition
                               (Section 2.3, Eqs. 6-8)
  * ``lpd``                 -- log pointwise predictive density of held-out
                               pairs (model selection, Section 2)
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mds_oracle.c")
_LIB_PATH = os.path.join(_HERE, "libmds_oracle.so")
_lib = None

_dp = ctypes.POINTER(ctypes.c_double)
_u8p = ctypes.POINTER(ctypes.c_ubyte)
_i64p = ctypes.POINTER(ctypes.c_int64)
_u32p = ctypes.POINTER(ctypes.c_uint32)


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, strict IEEE: no fast-math)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-fno-fast-math",
             "-ffp-contract=off", "-Wall", "-Wextra", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build(force=False)
    lib = ctypes.CDLL(_LIB_PATH)
    lib.oracle_log_phi.restype = ctypes.c_double
    lib.oracle_log_phi.argtypes = [ctypes.c_double]
    lib.oracle_mills.restype = ctypes.c_double
    lib.oracle_mills.argtypes = [ctypes.c_double]
    lib.oracle_count_observed.restype = ctypes.c_int64
    lib.oracle_count_observed.argtypes = [ctypes.c_int64, _dp, ctypes.c_int64, _u8p,
                                          ctypes.c_int64]
    lib.oracle_eval.restype = ctypes.c_int
    lib.oracle_eval.argtypes = [ctypes.c_int64, ctypes.c_int, _dp, ctypes.c_int64, _dp,
                                ctypes.c_int64, _u8p, ctypes.c_int64, ctypes.c_double,
                                _dp, _dp, _dp, _dp, _dp, _dp, _dp, _i64p]
    lib.oracle_lpd.restype = ctypes.c_int
    lib.oracle_lpd.argtypes = [ctypes.c_int64, ctypes.c_int, ctypes.c_int64, _dp, _dp, _dp,
                               ctypes.c_int64, _u8p, ctypes.c_int64, _dp, _i64p]
    lib.oracle_eval_normal.restype = ctypes.c_int
    lib.oracle_eval_normal.argtypes = lib.oracle_eval.argtypes
    lib.oracle_leapfrog.restype = ctypes.c_int
    lib.oracle_leapfrog.argtypes = [ctypes.c_int64, ctypes.c_int, _dp, _dp, _dp,
                                    ctypes.c_int64, _u8p, ctypes.c_int64, ctypes.c_double,
                                    _dp, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                    _dp, _dp, _dp, _dp, _dp, ctypes.c_int]
    lib.oracle_grad_rows_given.restype = ctypes.c_int
    lib.oracle_grad_rows_given.argtypes = [ctypes.c_int64, ctypes.c_int, _dp, ctypes.c_int64, _dp,
                                           ctypes.c_int64, ctypes.c_double, _i64p, ctypes.c_int64,
                                           _dp, _dp, _dp]
    lib.oracle_grad_rows.restype = ctypes.c_int
    lib.oracle_philox4x32_10.restype = None
    lib.oracle_philox4x32_10.argtypes = [_u32p, _u32p, _u32p]
    lib.oracle_uniform_open.restype = ctypes.c_double
    lib.oracle_uniform_open.argtypes = [ctypes.c_uint32, ctypes.c_uint32]
    lib.oracle_momentum.restype = None
    lib.oracle_momentum.argtypes = [ctypes.c_int64, ctypes.c_int, _dp, ctypes.c_uint64,
                                    ctypes.c_uint64, _dp]
    lib.oracle_accept_uniform.restype = ctypes.c_double
    lib.oracle_accept_uniform.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
    lib.oracle_hmc_step.restype = ctypes.c_int
    lib.oracle_hmc_step.argtypes = [ctypes.c_int64, ctypes.c_int, _dp, _dp, ctypes.c_int64, _u8p,
                                    ctypes.c_int64, ctypes.c_double, _dp, ctypes.c_double,
                                    ctypes.c_double, ctypes.c_int, ctypes.c_uint64,
                                    ctypes.c_uint64, _dp, _dp, _dp, _dp, _dp, _dp,
                                    ctypes.POINTER(ctypes.c_int), ctypes.c_int]
    lib.oracle_grad_rows.argtypes = [ctypes.c_int64, ctypes.c_int, _dp, ctypes.c_int64, _dp,
                                     ctypes.c_int64, _u8p, ctypes.c_int64, ctypes.c_double,
                                     _i64p, ctypes.c_int64, _dp, _dp, _dp]
    _lib = lib
    return lib


def _ptr(a, typ=_dp):
    if a is None:
        return None
    return a.ctypes.data_as(typ)


def _as_y(y):
    y = np.ascontiguousarray(y, dtype=np.float64)
    return y


def _as_mask(mask, n):
    if mask is None:
        return None
    m = np.ascontiguousarray(mask)
    if m.dtype != np.uint8:
        m = (m != 0).astype(np.uint8)
    assert m.shape == (n, n)
    return m


def log_phi(t) -> np.ndarray:
    """ln Phi(t) elementwise (any real t)."""
    lib = _load()
    t = np.asarray(t, dtype=np.float64)
    return np.vectorize(lib.oracle_log_phi, otypes=[np.float64])(t)


def mills(t) -> np.ndarray:
    """phi(t)/Phi(t) elementwise (any real t)."""
    lib = _load()
    t = np.asarray(t, dtype=np.float64)
    return np.vectorize(lib.oracle_mills, otypes=[np.float64])(t)


def count_observed(y, mask=None) -> int:
    lib = _load()
    y = _as_y(y)
    n = y.shape[0]
    m = _as_mask(mask, n)
    return int(lib.oracle_count_observed(n, _ptr(y), y.shape[1], _ptr(m, _u8p),
                                         n if m is not None else 0))


@dataclass
class Evaluation:
    loglik: float
    grad: np.ndarray      # N x D
    dsigma: float
    absrow: np.ndarray    # N: A_i = sum_j |w_ij|
    condrow: np.ndarray   # N: B_i = sum_j (delta+|y|)/sigma^2 + m/sigma, row rounding scale
    abs_loglik: float     # sum |r_ij| + M |ln sigma|
    abs_dsigma: float     # sum |d r_ij/d sigma| + M / sigma
    m_obs: int


def evaluate(x, y, sigma: float, mask=None, truncated: bool = True) -> Evaluation:
    """L, dL/dX and dL/dsigma of Eq. (2)/(9) at X for dissimilarities Y
    (truncated=False: the same model without the truncation to y > 0)."""
    lib = _load()
    x = np.ascontiguousarray(x, dtype=np.float64)
    if x.ndim == 1:
        x = x[:, None]
    n, d = x.shape
    y = _as_y(y)
    assert y.shape[0] == n and y.shape[1] >= n
    m = _as_mask(mask, n)
    grad = np.zeros((n, d), dtype=np.float64)
    absrow = np.zeros(n, dtype=np.float64)
    condrow = np.zeros(n, dtype=np.float64)
    out = (ctypes.c_double * 5)()
    mobs = ctypes.c_int64(0)
    fn = lib.oracle_eval if truncated else lib.oracle_eval_normal
    rc = fn(n, d, _ptr(x), d, _ptr(y), y.shape[1], _ptr(m, _u8p), n if m is not None else 0,
            float(sigma), ctypes.cast(ctypes.byref(out, 0), _dp), _ptr(grad),
            ctypes.cast(ctypes.byref(out, 8), _dp), _ptr(absrow), _ptr(condrow),
            ctypes.cast(ctypes.byref(out, 16), _dp), ctypes.cast(ctypes.byref(out, 24), _dp),
            ctypes.byref(mobs))
    if rc != 0:
        raise ValueError("oracle_eval rejected its arguments")
    return Evaluation(out[0], grad, out[1], absrow, condrow, out[2], out[3], int(mobs.value))


def grad_rows(x, y, sigma: float, rows, mask=None):
    """Gradient rows (Eq. 9) of the listed points only, with their A_i and B_i."""
    lib = _load()
    x = np.ascontiguousarray(x, dtype=np.float64)
    n, d = x.shape
    y = _as_y(y)
    m = _as_mask(mask, n)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    g = np.zeros((rows.size, d), dtype=np.float64)
    a = np.zeros(rows.size, dtype=np.float64)
    b = np.zeros(rows.size, dtype=np.float64)
    rc = lib.oracle_grad_rows(n, d, _ptr(x), d, _ptr(y), y.shape[1], _ptr(m, _u8p),
                              n if m is not None else 0, float(sigma), _ptr(rows, _i64p),
                              rows.size, _ptr(g), _ptr(a), _ptr(b))
    if rc != 0:
        raise ValueError("oracle_grad_rows rejected its arguments")
    return g, a, b


def grad_rows_given(x, yrows, sigma: float, rows):
    """Gradient rows (Eq. 9) of the listed points from their whole rows of the
    symmetric Y (len(rows) x N, NaN = missing), with A_i and B_i."""
    lib = _load()
    x = np.ascontiguousarray(x, dtype=np.float64)
    n, d = x.shape
    yr = np.ascontiguousarray(yrows, dtype=np.float64).reshape(-1, n)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    if yr.shape[0] != rows.size:
        raise ValueError("one Y row per listed point")
    g = np.zeros((rows.size, d), dtype=np.float64)
    a = np.zeros(rows.size, dtype=np.float64)
    b = np.zeros(rows.size, dtype=np.float64)
    rc = lib.oracle_grad_rows_given(n, d, _ptr(x), d, _ptr(yr), n, float(sigma),
                                    _ptr(rows, _i64p), rows.size, _ptr(g), _ptr(a), _ptr(b))
    if rc != 0:
        raise ValueError("oracle_grad_rows_given rejected its arguments")
    return g, a, b


@dataclass
class Trajectory:
    x: np.ndarray
    p: np.ndarray
    grad_end: np.ndarray
    loglik_start: float
    loglik_end: float
    energy_start: float
    energy_end: float


def leapfrog(x, p, y, sigma: float, eps: float, n_steps: int, mask=None,
             inv_mass=None, prior_precision: float = 0.0, truncated: bool = True) -> Trajectory:
    """One leapfrog trajectory (Section 2.3); returns copies, inputs untouched.
    ``truncated=False`` targets the model without the truncation to y > 0."""
    lib = _load()
    x = np.array(x, dtype=np.float64, copy=True, order="C")
    p = np.array(p, dtype=np.float64, copy=True, order="C")
    n, d = x.shape
    assert p.shape == (n, d)
    y = _as_y(y)
    m = _as_mask(mask, n)
    im = None if inv_mass is None else np.ascontiguousarray(inv_mass, dtype=np.float64)
    if im is not None:
        assert im.shape == (n, d)
    g = np.zeros((n, d), dtype=np.float64)
    out = (ctypes.c_double * 4)()
    rc = lib.oracle_leapfrog(n, d, _ptr(x), _ptr(p), _ptr(y), y.shape[1], _ptr(m, _u8p),
                             n if m is not None else 0, float(sigma), _ptr(im), float(eps),
                             float(prior_precision), int(n_steps), _ptr(g),
                             ctypes.cast(ctypes.byref(out, 0), _dp),
                             ctypes.cast(ctypes.byref(out, 8), _dp),
                             ctypes.cast(ctypes.byref(out, 16), _dp),
                             ctypes.cast(ctypes.byref(out, 24), _dp), 1 if truncated else 0)
    if rc != 0:
        raise ValueError("oracle_leapfrog rejected its arguments")
    return Trajectory(x, p, g, out[0], out[1], out[2], out[3])


# ------------------------------------------------------ HMC transition ----

def philox4x32_10(ctr, key):
    """The Philox4x32-10 block for a 4-word counter and a 2-word key."""
    lib = _load()
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib.oracle_philox4x32_10(_ptr(c, _u32p), _ptr(k, _u32p), _ptr(out, _u32p))
    return out


def uniform_open(a: int, b: int) -> float:
    return _load().oracle_uniform_open(int(a), int(b))


def momentum(n: int, d: int, seed: int, iteration: int, inv_mass=None) -> np.ndarray:
    """The momentum draw of HMC transition `iteration` (N x D)."""
    lib = _load()
    im = None if inv_mass is None else np.ascontiguousarray(inv_mass, dtype=np.float64)
    p = np.zeros((n, d), dtype=np.float64)
    lib.oracle_momentum(n, d, _ptr(im), int(seed), int(iteration), _ptr(p))
    return p


def accept_uniform(seed: int, iteration: int) -> float:
    return _load().oracle_accept_uniform(int(seed), int(iteration))


@dataclass
class HMCStep:
    x: np.ndarray
    p: np.ndarray
    grad: np.ndarray
    loglik: float
    energy_start: float
    energy_end: float
    log_u: float
    accepted: bool


def hmc_step(x, y, sigma: float, eps: float, n_steps: int, seed: int, iteration: int,
             mask=None, inv_mass=None, prior_precision: float = 0.0,
             truncated: bool = True) -> HMCStep:
    """One HMC transition (Section 2.3) from state x; inputs untouched."""
    lib = _load()
    x = np.array(x, dtype=np.float64, copy=True, order="C")
    n, d = x.shape
    y = _as_y(y)
    m = _as_mask(mask, n)
    im = None if inv_mass is None else np.ascontiguousarray(inv_mass, dtype=np.float64)
    p = np.zeros((n, d), dtype=np.float64)
    g = np.zeros((n, d), dtype=np.float64)
    out = (ctypes.c_double * 4)()
    acc = ctypes.c_int(0)
    rc = lib.oracle_hmc_step(n, d, _ptr(x), _ptr(y), y.shape[1], _ptr(m, _u8p),
                             n if m is not None else 0, float(sigma), _ptr(im), float(eps),
                             float(prior_precision), int(n_steps), int(seed), int(iteration),
                             _ptr(p), _ptr(g), ctypes.cast(ctypes.byref(out, 0), _dp),
                             ctypes.cast(ctypes.byref(out, 8), _dp),
                             ctypes.cast(ctypes.byref(out, 16), _dp),
                             ctypes.cast(ctypes.byref(out, 24), _dp), ctypes.byref(acc),
                             1 if truncated else 0)
    if rc != 0:
        raise ValueError("oracle_hmc_step rejected its arguments")
    return HMCStep(x, p, g, out[0], out[1], out[2], out[3], bool(acc.value))


def lpd(xs, sigmas, y, heldout, mask=None):
    """Log pointwise predictive density of the held-out pairs (heldout != 0,
    observed: mask zero and y not NaN) over the posterior draws xs (S x N x D,
    or one N x D state) and sigmas (S values); returns (lpd, pairs)."""
    lib = _load()
    xs = np.ascontiguousarray(xs, dtype=np.float64)
    if xs.ndim == 2:
        xs = xs[None]
    s_draws, n, d = xs.shape
    sig = np.ascontiguousarray(np.broadcast_to(np.asarray(sigmas, dtype=np.float64), (s_draws,)))
    y = _as_y(y)
    keep_out = np.asarray(heldout) == 0
    m = keep_out if mask is None else (keep_out | (np.asarray(mask) != 0))
    m = np.ascontiguousarray(m, dtype=np.uint8)
    out = ctypes.c_double(0.0)
    cnt = ctypes.c_int64(0)
    rc = lib.oracle_lpd(n, d, s_draws, _ptr(xs), _ptr(sig), _ptr(y), y.shape[1], _ptr(m, _u8p), n,
                        ctypes.byref(out), ctypes.byref(cnt))
    if rc != 0:
        raise ValueError("oracle_lpd rejected its arguments")
    return out.value, int(cnt.value)
