"""Thin ctypes binding of libmassivemds (include/massivemds.h).

Argument marshalling only: every step of the computation runs in the HIP
kernels of the library.  torch supplies device memory and the current stream.
If the library is missing the binding raises -- there is no CPU fallback.

Low-level functions carry the C names (``mds_loglik``, ``mds_gradient``,
``mds_leapfrog``, ``mds_prepare_y``, ``mds_spatial_order``, ``mds_permute_rows``,
``mds_log_phi``, ``mds_workspace_bytes``);
``MDSProblem`` bundles a prepared Y with its workspace.
"""
from __future__ import annotations

import ctypes
import os

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
# MDS_LIB_PATH may name another build of the same library (e.g. a variant)
LIB_PATH = os.environ.get("MDS_LIB_PATH", os.path.join(_PKG, "libmassivemds.so"))

MDS_OK = 0
MDS_UNTRUNCATED = 0x100      # model flag: no truncation to y > 0 (plain normal errors)
MDS_ERR_INVALID_ARGUMENT = -1
MDS_ERR_UNSUPPORTED = -2
MDS_ERR_WORKSPACE_TOO_SMALL = -3
MDS_ERR_HIP = -4
MDS_ERR_NOT_SYMMETRIC = -5
MDS_F64 = 0
MDS_F32 = 1
MDS_MAX_DIM = 8
WORKSPACE_ALIGN = 256
BATCH_DEFAULT_WAVES = 2      # the library's batch tile_waves when 0 is passed

_c_i64 = ctypes.c_int64
_c_i32 = ctypes.c_int32
_vp = ctypes.c_void_p
_lib = None


class ProblemDesc(ctypes.Structure):
    """mirror of mds_problem_desc"""
    _fields_ = [("n", _c_i64), ("d", _c_i32), ("tile_rows", _c_i32), ("x", _vp), ("ldx", _c_i64),
                ("y", _vp), ("ldy", _c_i64), ("sigma", _vp), ("scale", _vp), ("grad", _vp),
                ("ldg", _c_i64), ("loglik", _vp), ("dsigma", _vp), ("dlogsigma", _vp),
                ("p", _vp), ("ldp", _c_i64), ("step", _vp)]


class BatchPlan(ctypes.Structure):
    """mirror of mds_batch_plan"""
    _fields_ = [("count", _c_i32), ("y_dtype", _c_i32), ("tile_waves", _c_i32), ("grid", _c_i32),
                ("max_d", _c_i32), ("flags", _c_i32), ("total_tiles", _c_i64), ("elem_blocks", _c_i64), ("lds_bytes", ctypes.c_size_t),
                ("workspace", _vp), ("workspace_bytes", ctypes.c_size_t)]


class MDSError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str):
        super().__init__(f"{where} failed with {status}: {detail}")
        self.status = status


def lib():
    """Load libmassivemds.so (after torch, so both share one HIP runtime)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"{LIB_PATH} is not built: run `python -m paper_1905_04582_amd.build` "
            "(the MDS path has no CPU fallback)")
    L = ctypes.CDLL(LIB_PATH)
    L.mds_status_string.restype = ctypes.c_char_p
    L.mds_status_string.argtypes = [ctypes.c_int]
    L.mds_last_error.restype = ctypes.c_char_p
    L.mds_last_error.argtypes = []
    L.mds_version.restype = ctypes.c_int
    L.mds_workspace_bytes.restype = ctypes.c_int
    L.mds_workspace_bytes.argtypes = [_c_i64, _c_i32, _c_i32, _c_i32, _c_i32,
                                      ctypes.POINTER(ctypes.c_size_t)]
    L.mds_prepare_y.restype = ctypes.c_int
    L.mds_prepare_y.argtypes = [_vp, _c_i32, _c_i64, _vp, _c_i64, _vp, _c_i32, _c_i64, _c_i64,
                                _vp, _vp, _vp]
    L.mds_hmc_workspace_bytes.restype = ctypes.c_int
    L.mds_hmc_workspace_bytes.argtypes = [_c_i64, _c_i32, _c_i32, _c_i32, _c_i32,
                                          ctypes.POINTER(ctypes.c_size_t)]
    L.mds_hmc_momentum.restype = ctypes.c_int
    L.mds_hmc_momentum.argtypes = [_c_i64, _c_i32, _vp, ctypes.c_uint64, _vp, _vp, _c_i64, _vp]
    L.mds_hmc_step.restype = ctypes.c_int
    L.mds_hmc_step.argtypes = [_c_i64, _c_i32, _vp, _c_i64, _vp, _c_i32, _c_i64, _vp, _vp, _vp,
                               _vp, _c_i32, ctypes.c_uint64, _vp, _vp, _c_i64, _vp, _vp, _c_i32,
                               _vp, _vp, _vp, ctypes.c_size_t, _c_i32, _c_i32, _vp]
    L.mds_heldout_workspace_bytes.restype = ctypes.c_int
    L.mds_heldout_workspace_bytes.argtypes = [_c_i64, ctypes.POINTER(ctypes.c_size_t)]
    L.mds_heldout_count.restype = ctypes.c_int
    L.mds_heldout_count.argtypes = [_vp, _c_i32, _c_i64, _vp, _c_i64, _vp, _c_i64, _c_i64, _vp,
                                    _vp, ctypes.c_size_t, _vp]
    L.mds_heldout_fill.restype = ctypes.c_int
    L.mds_heldout_fill.argtypes = [_vp, _c_i32, _c_i64, _vp, _c_i64, _vp, _c_i64, _c_i64, _vp,
                                   ctypes.c_size_t, _c_i64, _vp, _vp, _vp, _vp]
    L.mds_lpd_accumulate.restype = ctypes.c_int
    L.mds_lpd_accumulate.argtypes = [_c_i64, _vp, _vp, _vp, _c_i32, _vp, _c_i64, _vp, _vp, _c_i32,
                                     _vp]
    L.mds_lpd_accumulate_draws.restype = ctypes.c_int
    L.mds_lpd_accumulate_draws.argtypes = [_c_i64, _vp, _vp, _vp, _c_i32, _vp, _c_i64, _c_i64,
                                           _vp, _c_i32, _vp, _c_i32, _vp]
    L.mds_lpd_finalize.restype = ctypes.c_int
    L.mds_lpd_finalize.argtypes = [_c_i64, _vp, _c_i64, _vp, ctypes.c_size_t, _vp, _vp]
    L.mds_lpd_workspace_bytes.restype = ctypes.c_int
    L.mds_lpd_workspace_bytes.argtypes = [_c_i64, ctypes.POINTER(ctypes.c_size_t)]
    L.mds_check_symmetric.restype = ctypes.c_int
    L.mds_check_symmetric.argtypes = [_vp, _c_i32, _c_i64, _c_i64, _vp, _vp]
    L.mds_require_symmetric.restype = ctypes.c_int
    L.mds_require_symmetric.argtypes = [_vp, _c_i32, _c_i64, _c_i64, _vp, _vp]
    L.mds_resolve_tiling.restype = ctypes.c_int
    L.mds_resolve_tiling.argtypes = [_c_i64, _c_i32, _c_i32, _c_i32, _c_i32,
                                     ctypes.POINTER(_c_i32), ctypes.POINTER(_c_i32)]
    L.mds_order_workspace_bytes.restype = ctypes.c_int
    L.mds_order_workspace_bytes.argtypes = [_c_i64, ctypes.POINTER(ctypes.c_size_t)]
    L.mds_spatial_order.restype = ctypes.c_int
    L.mds_spatial_order.argtypes = [_c_i64, _c_i32, _vp, _c_i64, _vp, _vp, ctypes.c_size_t, _vp]
    L.mds_permute_rows.restype = ctypes.c_int
    L.mds_permute_rows.argtypes = [_c_i64, _c_i32, _vp, _c_i64, _vp, _c_i64, _vp, _c_i32, _vp]
    L.mds_loglik.restype = ctypes.c_int
    L.mds_loglik.argtypes = [_c_i64, _c_i32, _vp, _c_i64, _vp, _c_i32, _c_i64, _vp, _vp, _vp,
                             ctypes.c_size_t, _c_i32, _c_i32, _vp]
    L.mds_gradient.restype = ctypes.c_int
    L.mds_gradient.argtypes = [_c_i64, _c_i32, _vp, _c_i64, _vp, _c_i32, _c_i64, _vp, _vp, _vp,
                               _c_i64, _vp, _vp, _vp, _vp, ctypes.c_size_t, _c_i32, _c_i32,
                               _vp]
    L.mds_noalloc_scratch_bytes.restype = ctypes.c_size_t
    L.mds_noalloc_scratch_bytes.argtypes = []
    L.mds_gradient_noalloc.restype = ctypes.c_int
    L.mds_gradient_noalloc.argtypes = [_c_i64, _c_i32, _vp, _c_i64, _vp, _c_i32, _c_i64, _vp, _vp,
                                       _vp, _c_i64, _vp, _vp, _vp, _c_i32, _c_i32, _vp]
    L.mds_leapfrog.restype = ctypes.c_int
    L.mds_leapfrog.argtypes = [_c_i64, _c_i32, _vp, _c_i64, _vp, _c_i64, _vp, _c_i32, _c_i64,
                               _vp, _vp, _vp, _vp, _c_i32, _vp, _vp, _c_i32, _vp, _vp, _vp,
                               ctypes.c_size_t, _c_i32, _c_i32, _vp]
    L.mds_log_phi.restype = ctypes.c_int
    L.mds_log_phi.argtypes = [_vp, _vp, _vp, _c_i64, _c_i32, _vp]
    L.mds_set_sweep_events.restype = ctypes.c_int
    L.mds_set_sweep_events.argtypes = [_vp, _vp]
    L.mds_set_tile_trace.restype = ctypes.c_int
    L.mds_set_tile_trace.argtypes = [_vp]
    L.mds_batch_workspace_bytes.restype = ctypes.c_int
    L.mds_batch_workspace_bytes.argtypes = [ctypes.POINTER(ProblemDesc), _c_i32, _c_i32, _c_i32,
                                            ctypes.POINTER(ctypes.c_size_t)]
    L.mds_batch_init.restype = ctypes.c_int
    L.mds_batch_init.argtypes = [ctypes.POINTER(ProblemDesc), _c_i32, _c_i32, _c_i32, _vp,
                                 ctypes.c_size_t, ctypes.POINTER(BatchPlan), _vp]
    L.mds_batch_eval.restype = ctypes.c_int
    L.mds_batch_eval.argtypes = [ctypes.POINTER(BatchPlan), _c_i32, _vp]
    L.mds_batch_leapfrog.restype = ctypes.c_int
    L.mds_batch_leapfrog.argtypes = [ctypes.POINTER(BatchPlan), _c_i32, _c_i32, _vp]
    _lib = L
    return L


def _check(status: int, where: str):
    if status != MDS_OK:
        L = lib()
        raise MDSError(status, where, f"{L.mds_status_string(status).decode()}: "
                                      f"{L.mds_last_error().decode()}")


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream=None, *tensors):
    """The raw stream a call is enqueued on.  When the caller names a stream,
    every device tensor the call hands to a kernel (temporaries included:
    converted inputs, device scalars made from numbers, fresh outputs) is
    recorded on it, so that the caching allocator does not hand its memory
    out again before the kernel has run."""
    s = torch.cuda.current_stream() if stream is None else stream
    if stream is not None:
        for t in tensors:
            if isinstance(t, torch.Tensor) and t.is_cuda:
                t.record_stream(stream)
    return ctypes.c_void_p(s.cuda_stream)


def _ycode(y, truncated: bool) -> int:
    return _dtype_code(y.dtype) | (0 if truncated else MDS_UNTRUNCATED)


def _dtype_code(dt: torch.dtype) -> int:
    if dt == torch.float64:
        return MDS_F64
    if dt == torch.float32:
        return MDS_F32
    raise TypeError(f"unsupported dtype {dt}: Y is float64 or float32")


def _dev_scalar(v, device):
    if isinstance(v, torch.Tensor):
        if v.dtype != torch.float64 or v.numel() != 1 or not v.is_cuda:
            raise TypeError("device scalars are 1-element float64 CUDA tensors")
        return v
    return torch.tensor(float(v), dtype=torch.float64, device=device)


def _check_mat(t, name, dtype=torch.float64):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if t.dim() != 2 or (t.numel() > 0 and t.shape[1] > 1 and t.stride(1) != 1):
        raise ValueError(f"{name} must be 2-D with unit column stride")


def _ld(t) -> int:
    """Leading dimension of a 2-D tensor; torch reports 0 for empty ones."""
    if t.shape[0] <= 1:
        return max(int(t.stride(0)), int(t.shape[1]), 1)
    return int(t.stride(0))


def version() -> int:
    return lib().mds_version()


def mds_workspace_bytes(n: int, d: int, y_dtype: int, tile_rows: int = 0,
                        tile_waves: int = 0) -> int:
    out = ctypes.c_size_t(0)
    _check(lib().mds_workspace_bytes(n, d, y_dtype, tile_rows, tile_waves, ctypes.byref(out)),
           "mds_workspace_bytes")
    return int(out.value)


def tile_waves(wc: int, wr: int = 1) -> int:
    """The tile_waves argument: wc 64-column waves across a tile, wr waves
    down its rows (MDS_TILE_WAVES)."""
    return int(wc) | (int(wr) << 8) if wr != 1 else int(wc)


def split_tile_waves(tw: int):
    """(column waves, row waves) of a tile_waves value."""
    wr = (int(tw) >> 8) & 0xFF
    return int(tw) & 0xFF, (wr if wr else 1)


def mds_resolve_tiling(n: int, d: int, y_dtype: int, tile_rows: int = 0,
                       tile_waves: int = 0):
    """(rows per tile, tile_waves) the sweeps use; tile_waves is the plain
    column-wave count when the tile's waves do not split its rows (see
    ``split_tile_waves``)."""
    r, w = _c_i32(), _c_i32()
    _check(lib().mds_resolve_tiling(n, d, y_dtype, tile_rows, tile_waves, ctypes.byref(r),
                                    ctypes.byref(w)), "mds_resolve_tiling")
    return r.value, w.value


def alloc_workspace(nbytes: int, device) -> torch.Tensor:
    ws = torch.empty(max(int(nbytes), WORKSPACE_ALIGN) + WORKSPACE_ALIGN, dtype=torch.uint8,
                     device=device)
    off = (-ws.data_ptr()) % WORKSPACE_ALIGN
    return ws[off:off + max(int(nbytes), WORKSPACE_ALIGN)]


def padded_ld(n: int) -> int:
    """Leading dimension of prepared Y: N rounded up to 64 elements."""
    return max(64, (n + 63) // 64 * 64)


def mds_prepare_y(y_src: torch.Tensor, out_dtype: torch.dtype = torch.float64, mask=None,
                  ldy: int | None = None, count: bool = True, perm=None, stream=None):
    """Y -> device Y' in out_dtype with missing entries folded into NaN,
    relabelled by ``perm`` (Y'[k, l] = Y[perm[k], perm[l]]) when given.
    Returns (y_prepared N x ldy view, m_obs device int64 tensor or None)."""
    _check_mat(y_src, "y_src", y_src.dtype)
    if perm is not None:
        _check_perm(perm, y_src.shape[0], y_src.device)
    n = y_src.shape[0]
    if y_src.shape[1] < n:
        raise ValueError("y_src must be N x N")
    ldy = padded_ld(n) if ldy is None else int(ldy)
    buf = torch.empty((max(n, 1), ldy), dtype=out_dtype, device=y_src.device)
    if mask is not None:
        _check_mat(mask, "mask", torch.uint8)
    m_obs = torch.zeros((), dtype=torch.int64, device=y_src.device) if count else None
    _check(lib().mds_prepare_y(_ptr(y_src), _dtype_code(y_src.dtype), _ld(y_src),
                               _ptr(mask), _ld(mask) if mask is not None else 0,
                               _ptr(buf), _dtype_code(out_dtype), ldy, n, _ptr(perm),
                               _ptr(m_obs), _stream(stream, y_src, mask, buf, perm, m_obs)), "mds_prepare_y")
    return buf[:n], m_obs


def mds_check_symmetric(y: torch.Tensor, stream=None) -> int:
    """Number of pairs i > j with y[i, j] != y[j, i] (two NaNs count as equal);
    synchronises to read the count."""
    _check_mat(y, "y", y.dtype)
    n = y.shape[0]
    cnt = torch.zeros((), dtype=torch.int64, device=y.device)
    _check(lib().mds_check_symmetric(_ptr(y), _dtype_code(y.dtype), _ld(y), n, _ptr(cnt),
                                     _stream(stream, y, cnt)), "mds_check_symmetric")
    return int(cnt.item())


def mds_require_symmetric(y: torch.Tensor, stream=None):
    """The library's checked mode: raises MDSError(MDS_ERR_NOT_SYMMETRIC) when
    some pair i > j has y[i, j] != y[j, i] (two NaNs count as equal);
    synchronises."""
    _check_mat(y, "y", y.dtype)
    n = y.shape[0]
    cnt = torch.zeros((), dtype=torch.int64, device=y.device)
    _check(lib().mds_require_symmetric(_ptr(y), _dtype_code(y.dtype), _ld(y), n, _ptr(cnt),
                                       _stream(stream, y, cnt)), "mds_require_symmetric")


def _check_perm(perm, n, device):
    if not (isinstance(perm, torch.Tensor) and perm.dtype == torch.int64 and perm.is_contiguous()
            and perm.dim() == 1 and perm.numel() == n and perm.device == torch.device(device)):
        raise ValueError("perm must be a contiguous int64 device tensor of length N")


def mds_spatial_order(x: torch.Tensor, stream=None) -> torch.Tensor:
    """Locality-preserving order of the rows of x (Hilbert curve for D = 2,
    Morton order otherwise): perm[k] = original index of the k-th location."""
    _check_mat(x, "x")
    n, d = x.shape
    nb = ctypes.c_size_t()
    _check(lib().mds_order_workspace_bytes(n, ctypes.byref(nb)), "mds_order_workspace_bytes")
    ws = alloc_workspace(nb.value, x.device)
    perm = torch.empty(max(n, 1), dtype=torch.int64, device=x.device)[:n]
    _check(lib().mds_spatial_order(n, d, _ptr(x), _ld(x), _ptr(perm), _ptr(ws), nb.value,
                                   _stream(stream, x, perm, ws)), "mds_spatial_order")
    return perm


def mds_permute_rows(src: torch.Tensor, perm: torch.Tensor, inverse: bool = False, out=None,
                     stream=None) -> torch.Tensor:
    """out[k] = src[perm[k]] (inverse=False) or out[perm[k]] = src[k] (inverse=True)."""
    _check_mat(src, "src")
    n, d = src.shape
    _check_perm(perm, n, src.device)
    out = torch.empty_like(src) if out is None else out
    _check_mat(out, "out")
    _check(lib().mds_permute_rows(n, d, _ptr(src), _ld(src), _ptr(out), _ld(out), _ptr(perm),
                                  1 if inverse else 0, _stream(stream, src, perm, out)), "mds_permute_rows")
    return out


def mds_loglik(x, y, sigma, workspace, out=None, tile_rows=0, tile_waves=0, stream=None,
               truncated=True):
    _check_mat(x, "x")
    _check_mat(y, "y", y.dtype)
    n, d = x.shape
    sig = _dev_scalar(sigma, x.device)
    out = torch.empty((), dtype=torch.float64, device=x.device) if out is None else out
    _check(lib().mds_loglik(n, d, _ptr(x), _ld(x), _ptr(y), _ycode(y, truncated),
                            _ld(y), _ptr(sig), _ptr(out), _ptr(workspace),
                            workspace.numel(), tile_rows, tile_waves,
                            _stream(stream, x, y, sig, out, workspace)),
           "mds_loglik")
    return out


def mds_gradient(x, y, sigma, workspace, scale=None, grad=None, loglik=None, dsigma=None,
                 want_loglik=True, want_dsigma=True, dlogsigma=None, tile_rows=0, tile_waves=0,
                 stream=None, truncated=True):
    """Returns (grad N x D, loglik scalar or None, dsigma scalar or None); an
    optional `dlogsigma` device scalar receives scale * sigma * dL/dsigma."""
    _check_mat(x, "x")
    _check_mat(y, "y", y.dtype)
    n, d = x.shape
    dev = x.device
    sig = _dev_scalar(sigma, dev)
    sc = None if scale is None else _dev_scalar(scale, dev)
    grad = torch.empty((n, d), dtype=torch.float64, device=dev) if grad is None else grad
    _check_mat(grad, "grad")
    if want_loglik and loglik is None:
        loglik = torch.empty((), dtype=torch.float64, device=dev)
    if want_dsigma and dsigma is None:
        dsigma = torch.empty((), dtype=torch.float64, device=dev)
    _check(lib().mds_gradient(n, d, _ptr(x), _ld(x), _ptr(y), _ycode(y, truncated),
                              _ld(y), _ptr(sig), _ptr(sc), _ptr(grad), _ld(grad),
                              _ptr(loglik), _ptr(dsigma), _ptr(dlogsigma), _ptr(workspace),
                              workspace.numel(), tile_rows, tile_waves,
                              _stream(stream, x, y, sig, sc, grad, loglik, dsigma, dlogsigma,
                                      workspace)),
           "mds_gradient")
    return grad, loglik, dsigma


def mds_gradient_noalloc(x, y, sigma, grad, loglik=None, dsigma=None, dlogsigma=None,
                         scale=None, tile_rows=0, tile_waves=0, stream=None, truncated=True):
    """mds_gradient without a workspace: the library's static device scratch
    holds the partial sums (see include/massivemds.h).  Every tensor is the
    caller's; sigma and scale must already be device scalars, so the call
    itself allocates nothing."""
    _check_mat(x, "x")
    _check_mat(y, "y", y.dtype)
    _check_mat(grad, "grad")
    n, d = x.shape
    for t, nm in ((sigma, "sigma"), (scale, "scale")):
        if t is not None and not (isinstance(t, torch.Tensor) and t.is_cuda and
                                  t.dtype == torch.float64 and t.numel() == 1):
            raise TypeError(f"{nm} must be a one-element float64 device tensor")
    _check(lib().mds_gradient_noalloc(n, d, _ptr(x), _ld(x), _ptr(y), _ycode(y, truncated),
                                      _ld(y), _ptr(sigma), _ptr(scale), _ptr(grad), _ld(grad),
                                      _ptr(loglik), _ptr(dsigma), _ptr(dlogsigma), tile_rows,
                                      tile_waves, _stream(stream, x, y, sigma, scale, grad, loglik,
                                                          dsigma, dlogsigma)),
           "mds_gradient_noalloc")
    return grad, loglik, dsigma


def mds_leapfrog(x, p, y, sigma, step, n_steps, workspace, grad_io, loglik_io,
                 cache_valid=False, inv_mass=None, prior=None, energy_start=None,
                 energy_end=None, tile_rows=0, tile_waves=0, stream=None, truncated=True):
    """In-place leapfrog trajectory on (x, p); grad_io/loglik_io are the
    gradient/log-likelihood cache at x (read if cache_valid, always written)."""
    for t, nm in ((x, "x"), (p, "p"), (grad_io, "grad_io")):
        _check_mat(t, nm)
    _check_mat(y, "y", y.dtype)
    n, d = x.shape
    if grad_io.shape != (n, d) or not grad_io.is_contiguous():
        raise ValueError("grad_io must be a contiguous N x D float64 tensor")
    if inv_mass is not None and (inv_mass.shape != (n, d) or not inv_mass.is_contiguous()
                                 or inv_mass.dtype != torch.float64):
        raise ValueError("inv_mass must be a contiguous N x D float64 tensor")
    dev = x.device
    sig = _dev_scalar(sigma, dev)
    eps = _dev_scalar(step, dev)
    lam = None if prior is None else _dev_scalar(prior, dev)
    _check(lib().mds_leapfrog(n, d, _ptr(x), _ld(x), _ptr(p), _ld(p), _ptr(y),
                              _ycode(y, truncated), _ld(y), _ptr(sig), _ptr(inv_mass),
                              _ptr(eps), _ptr(lam), int(n_steps), _ptr(grad_io), _ptr(loglik_io),
                              1 if cache_valid else 0, _ptr(energy_start), _ptr(energy_end),
                              _ptr(workspace), workspace.numel(), tile_rows, tile_waves,
                              _stream(stream, x, p, y, sig, inv_mass, eps, lam, grad_io, loglik_io,
                                      energy_start, energy_end, workspace)), "mds_leapfrog")


def mds_hmc_workspace_bytes(n: int, d: int, y_dtype: int, tile_rows: int = 0,
                            tile_waves: int = 0) -> int:
    nb = ctypes.c_size_t()
    _check(lib().mds_hmc_workspace_bytes(n, d, y_dtype, tile_rows, tile_waves, ctypes.byref(nb)),
           "mds_hmc_workspace_bytes")
    return int(nb.value)


def _check_counter(t, device):
    if not (isinstance(t, torch.Tensor) and t.dtype == torch.int64 and t.numel() == 1
            and t.device == torch.device(device)):
        raise ValueError("the transition counter must be a one-element int64 device tensor")


def mds_hmc_momentum(n: int, d: int, seed: int, iteration: torch.Tensor, inv_mass=None,
                     out=None, stream=None) -> torch.Tensor:
    """The momentum draw of HMC transition *iteration (an int64 device scalar
    read as uint64) under `seed`."""
    dev = iteration.device
    _check_counter(iteration, dev)
    out = torch.empty((n, d), dtype=torch.float64, device=dev) if out is None else out
    _check_mat(out, "out")
    if inv_mass is not None:
        _check_mat(inv_mass, "inv_mass")
    _check(lib().mds_hmc_momentum(n, d, _ptr(inv_mass), int(seed) & 0xFFFFFFFFFFFFFFFF,
                                  _ptr(iteration), _ptr(out), _ld(out),
                                  _stream(stream, inv_mass, iteration, out)),
           "mds_hmc_momentum")
    return out


def mds_hmc_step(x, p, y, sigma, step, n_steps, seed, iteration, workspace, grad_io, loglik_io,
                 cache_valid=False, inv_mass=None, prior=None, stats=None, accepted_total=None,
                 tile_rows=0, tile_waves=0, stream=None, truncated=True):
    """One HMC transition of the chain at x (in place); see include/massivemds.h."""
    for t, nm in ((x, "x"), (p, "p"), (grad_io, "grad_io")):
        _check_mat(t, nm)
    _check_mat(y, "y", y.dtype)
    n, d = x.shape
    dev = x.device
    _check_counter(iteration, dev)
    if grad_io.shape != (n, d) or not grad_io.is_contiguous():
        raise ValueError("grad_io must be a contiguous N x D float64 tensor")
    if inv_mass is not None and (inv_mass.shape != (n, d) or not inv_mass.is_contiguous()
                                 or inv_mass.dtype != torch.float64):
        raise ValueError("inv_mass must be a contiguous N x D float64 tensor")
    if stats is not None and (stats.dtype != torch.float64 or stats.numel() < 4):
        raise ValueError("stats must hold four float64 values")
    if accepted_total is not None:
        _check_counter(accepted_total, dev)
    sig = _dev_scalar(sigma, dev)
    eps = _dev_scalar(step, dev)
    lam = None if prior is None else _dev_scalar(prior, dev)
    _check(lib().mds_hmc_step(n, d, _ptr(x), _ld(x), _ptr(y), _ycode(y, truncated), _ld(y),
                              _ptr(sig), _ptr(inv_mass), _ptr(eps), _ptr(lam), int(n_steps),
                              int(seed) & 0xFFFFFFFFFFFFFFFF, _ptr(iteration), _ptr(p), _ld(p),
                              _ptr(grad_io), _ptr(loglik_io), 1 if cache_valid else 0,
                              _ptr(stats), _ptr(accepted_total), _ptr(workspace),
                              workspace.numel(), tile_rows, tile_waves,
                              _stream(stream, x, p, y, sig, inv_mass, eps, lam, iteration,
                                      grad_io, loglik_io, stats, accepted_total, workspace)),
           "mds_hmc_step")


def mds_log_phi(t: torch.Tensor, precision: int = MDS_F64, stream=None):
    """(ln Phi(t), phi(t)/Phi(t)) elementwise on the device."""
    if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous():
        raise TypeError("t must be a contiguous float64 device tensor")
    ln = torch.empty_like(t)
    mi = torch.empty_like(t)
    _check(lib().mds_log_phi(_ptr(t), _ptr(ln), _ptr(mi), t.numel(), precision,
                             _stream(stream, t, ln, mi)), "mds_log_phi")
    return ln, mi


def mds_set_sweep_events(before, after):
    """Bracket every later sweep launch of this thread with two raw hipEvent_t
    handles (ints), or stop with (None, None).  Benchmark diagnostics only."""
    _check(lib().mds_set_sweep_events(before, after), "mds_set_sweep_events")


def mds_set_tile_trace(buf):
    """Record every later single-problem sweep's per-wave (start clock, end
    clock, hardware slot) in ``buf`` (a uint64/int64 device tensor of
    tiles * waves * 3 entries), or stop with None.  Diagnostics only."""
    _check(lib().mds_set_tile_trace(None if buf is None else ctypes.c_void_p(buf.data_ptr())),
           "mds_set_tile_trace")


def tile_count(n: int, tile_rows: int, wc: int) -> int:
    """Work-groups of one sweep: tiles of tile_rows x 64*wc over the lower
    triangle of an n x n matrix."""
    br, cw = int(tile_rows), 64 * int(wc)
    nrb = (int(n) + br - 1) // br
    if br >= cw:
        k = br // cw
        return k * nrb * (nrb + 1) // 2
    k = cw // br
    a, b = divmod(nrb, k)
    return nrb + k * a * (a - 1) // 2 + a * b


class MDSProblem:
    """A prepared dissimilarity matrix on the device plus its workspace.

    y      N x N (numpy or torch, any device), symmetric
    mask   optional N x N, non-zero = missing
    dtype  torch.float64 (FP64 form) or torch.float32 (FP32 form)
    truncated  False: the model without the truncation to y > 0 (plain
           normal errors; the paper's comparison of the two)
    order  optional N x D locations (e.g. the chain's starting X): the problem
           is stored relabelled in their spatial order (``perm``), and every
           X, P and gradient passed to its methods is in that labelling --
           ``relabel`` / ``unlabel`` convert N x D arrays to and from it.
    """

    def __init__(self, y, d: int, mask=None, dtype=torch.float64, device="cuda",
                 tile_rows: int = 0, tile_waves: int = 0, autotuned: bool = False, order=None,
                 check_symmetric: bool = False, truncated: bool = True):
        y = torch.as_tensor(y)
        n = y.shape[0]
        if autotuned and tile_rows == 0 and tile_waves == 0:
            from . import autotune
            tile_rows, tile_waves = autotune.lookup(dtype, int(d), n, device)
        src = y.to(device=device, dtype=torch.float64 if y.dtype == torch.float64 else
                   torch.float32).contiguous()
        m = None
        if mask is not None:
            m = (torch.as_tensor(mask) != 0).to(device=device, dtype=torch.uint8).contiguous()
        self.n, self.d, self.dtype, self.device = n, int(d), dtype, torch.device(device)
        self.truncated = bool(truncated)
        self.perm = None
        if order is not None:
            xo = torch.as_tensor(order).to(device=device, dtype=torch.float64).contiguous()
            self.perm = mds_spatial_order(xo)
        self.y, self.m_obs = mds_prepare_y(src, dtype, m, perm=self.perm)
        if check_symmetric:
            mds_require_symmetric(self.y)
        del src, m
        self.tile_rows, self.tile_waves = tile_rows, tile_waves
        self.ws_bytes = mds_workspace_bytes(n, self.d, _dtype_code(dtype), tile_rows, tile_waves)
        self.workspace = alloc_workspace(self.ws_bytes, self.device)

    def relabel(self, a, out=None, stream=None):
        """N x D array in the caller's labelling -> the problem's labelling."""
        a = torch.as_tensor(a).to(device=self.device, dtype=torch.float64).contiguous()
        return a.clone() if self.perm is None else mds_permute_rows(a, self.perm, False, out,
                                                                    stream)

    def unlabel(self, a, out=None, stream=None):
        """N x D array in the problem's labelling -> the caller's labelling."""
        return a.clone() if self.perm is None else mds_permute_rows(a, self.perm, True, out,
                                                                    stream)

    def hmc_step(self, x, p, sigma, step, n_steps, seed, iteration, grad_io, loglik_io,
                 cache_valid=False, inv_mass=None, prior=None, stats=None, accepted_total=None,
                 stream=None):
        """One HMC transition (see ``mds_hmc_step``); x, p, grad_io in this
        problem's labelling."""
        nb = mds_hmc_workspace_bytes(self.n, self.d, _dtype_code(self.dtype), self.tile_rows,
                                     self.tile_waves)
        if getattr(self, "_hmc_ws", None) is None or self._hmc_ws.numel() < nb:
            self._hmc_ws = alloc_workspace(nb, self.device)
        mds_hmc_step(x, p, self.y, sigma, step, n_steps, seed, iteration, self._hmc_ws, grad_io,
                     loglik_io, cache_valid, inv_mass, prior, stats, accepted_total,
                     self.tile_rows, self.tile_waves, stream, self.truncated)

    def set_tiling(self, tile_rows: int, tile_waves: int):
        nb = mds_workspace_bytes(self.n, self.d, _dtype_code(self.dtype), tile_rows, tile_waves)
        if nb > self.workspace.numel():
            self.workspace = alloc_workspace(nb, self.device)
        self.tile_rows, self.tile_waves, self.ws_bytes = tile_rows, tile_waves, nb

    def loglik(self, x, sigma, out=None, stream=None):
        return mds_loglik(x, self.y, sigma, self.workspace, out, self.tile_rows,
                          self.tile_waves, stream, self.truncated)

    def gradient(self, x, sigma, scale=None, grad=None, loglik=None, dsigma=None,
                 want_loglik=True, want_dsigma=True, dlogsigma=None, stream=None):
        return mds_gradient(x, self.y, sigma, self.workspace, scale, grad, loglik, dsigma,
                            want_loglik, want_dsigma, dlogsigma, tile_rows=self.tile_rows,
                            tile_waves=self.tile_waves, stream=stream, truncated=self.truncated)

    def leapfrog(self, x, p, sigma, step, n_steps, grad_io, loglik_io, cache_valid=False,
                 inv_mass=None, prior=None, energy_start=None, energy_end=None, stream=None):
        mds_leapfrog(x, p, self.y, sigma, step, n_steps, self.workspace, grad_io, loglik_io,
                     cache_valid, inv_mass, prior, energy_start, energy_end, self.tile_rows,
                     self.tile_waves, stream, self.truncated)


class MDSBatch:
    """Independent problems evaluated together: one persistent sweep launch and
    one finalize launch per ``eval()``.

    problems  list of dicts {"y": N x N, "d": D, "mask": optional, "tile_rows": 0}
    dtype     Y storage/arithmetic (float32 or float64), common to the batch

    The batch owns static device buffers that the kernels read and write:
    ``x[k]`` (N_k x D_k, write your positions there), ``grad[k]``, the
    momenta ``p[k]`` of ``leapfrog``, and the per-problem scalars ``sigma``,
    ``scale``, ``loglik``, ``dsigma``, ``dlogsigma`` and ``step`` (float64
    tensors of length count).

    A problem dict may carry ``order`` (N x D locations, e.g. the starting
    X): that problem is then stored relabelled in their spatial order
    (``perm[k]``), and x[k], p[k], grad[k] are in that labelling --
    ``relabel(k, a)`` / ``unlabel(k, a)`` convert N x D arrays.
    """

    def __init__(self, problems, dtype=torch.float32, device="cuda", tile_waves: int = 0,
                 stream=None, autotuned: bool = False, truncated: bool = True):
        self.device = torch.device(device)
        if autotuned:
            problems, tile_waves = _autotuned_batch(problems, dtype, device, tile_waves)
        self.tile_waves = tile_waves  # common to the batch (0 = the library's default)
        self.dtype = dtype
        f64 = dict(dtype=torch.float64, device=self.device)
        count = len(problems)
        self.count = count
        self.ys, self.m_obs, self.x, self.grad, self.perm = [], [], [], [], []
        self.tiles = []  # (rows, 64-column groups) of each problem's tiles
        self._scal = torch.zeros((6, count), **f64)
        self.sigma, self.scale, self.loglik, self.dsigma, self.dlogsigma, self.step = self._scal
        self.sigma.fill_(1.0)
        self.scale.fill_(1.0)
        self.step.fill_(1e-3)
        self.p = []
        descs = (ProblemDesc * count)()
        for k, pr in enumerate(problems):
            y = torch.as_tensor(pr["y"])
            src = y.to(device=self.device, dtype=torch.float64 if y.dtype == torch.float64
                       else torch.float32).contiguous()
            m = pr.get("mask")
            if m is not None:
                m = (torch.as_tensor(m) != 0).to(device=self.device, dtype=torch.uint8).contiguous()
            perm = None
            if pr.get("order") is not None:
                xo = torch.as_tensor(pr["order"]).to(device=self.device,
                                                     dtype=torch.float64).contiguous()
                perm = mds_spatial_order(xo, stream=stream)
            self.perm.append(perm)
            yp, mo = mds_prepare_y(src, dtype, m, perm=perm, stream=stream)
            del src, m
            n, d = y.shape[0], int(pr["d"])
            xk = torch.zeros((n, d), **f64)
            gk = torch.zeros((n, d), **f64)
            pk = torch.zeros((n, d), **f64)
            self.ys.append(yp)
            self.m_obs.append(mo)
            self.x.append(xk)
            self.grad.append(gk)
            self.p.append(pk)
            q = descs[k]
            q.n, q.d, q.tile_rows = n, d, int(pr.get("tile_rows", 0))
            q.x, q.ldx = xk.data_ptr(), max(d, 1)
            q.y, q.ldy = yp.data_ptr(), _ld(yp)
            q.sigma = self.sigma.data_ptr() + 8 * k
            q.scale = self.scale.data_ptr() + 8 * k
            q.grad, q.ldg = gk.data_ptr(), max(d, 1)
            q.loglik = self.loglik.data_ptr() + 8 * k
            q.dsigma = self.dsigma.data_ptr() + 8 * k
            q.dlogsigma = self.dlogsigma.data_ptr() + 8 * k
            q.p, q.ldp = pk.data_ptr(), max(d, 1)
            q.step = self.step.data_ptr() + 8 * k
        self._descs = descs
        self._code = _dtype_code(dtype) | (0 if truncated else MDS_UNTRUNCATED)
        self._plan_tiles(tile_waves, stream)

    def _plan_tiles(self, tile_waves, stream=None):
        """Resolve every problem's tiling under the common tile_waves and
        (re)build the batch plan and its workspace (``mds_batch_init``)."""
        descs, count = self._descs, self.count
        self.tile_waves = tile_waves
        self.tiles = []
        for k in range(count):
            q = descs[k]
            code, waves = _dtype_code(self.dtype), tile_waves or BATCH_DEFAULT_WAVES
            if q.tile_rows == 0:
                try:
                    t = mds_resolve_tiling(q.n, q.d, code, 128, waves)
                except MDSError:
                    t = mds_resolve_tiling(q.n, q.d, code, 0, waves)
            else:
                t = mds_resolve_tiling(q.n, q.d, code, q.tile_rows, waves)
            self.tiles.append(t)
        nb = ctypes.c_size_t(0)
        _check(lib().mds_batch_workspace_bytes(descs, count, self._code, tile_waves,
                                               ctypes.byref(nb)), "mds_batch_workspace_bytes")
        self.workspace = alloc_workspace(int(nb.value), self.device)
        self.plan = BatchPlan()
        _check(lib().mds_batch_init(descs, count, self._code, tile_waves, _ptr(self.workspace),
                                    self.workspace.numel(), ctypes.byref(self.plan),
                                    _stream(stream)), "mds_batch_init")

    def retile(self, tile_waves: int = 0, rows=None, stream=None):
        """New tiles for the batch without preparing Y again: a common
        tile_waves and each problem's tile_rows (a list; None or 0 = the
        library's batch default).  The gradient, x, p and sigma buffers are
        kept; the workspace is replaced."""
        torch.cuda.synchronize(self.device)
        for k in range(self.count):
            self._descs[k].tile_rows = int(rows[k]) if rows is not None and rows[k] else 0
        self._plan_tiles(tile_waves, stream)

    def autotune(self, reps: int = 5, path: str | None = None):
        """Pick the batch's tiles by timing whole evaluations of this batch
        (``autotune.tune_batch_plan``): the library default, the plan from
        the batch tuner's cache, and every common wave layout with the
        cache's row tiles or uniform 128-row tiles.  Call it once x and sigma
        hold representative values (the cost of a tile depends on how many
        of its wavefronts skip the truncation terms).  Returns the timings."""
        from . import autotune
        return autotune.tune_batch_plan(self, reps=reps, path=path)

    def set_x(self, k, x):
        """x in the problem's own (original) labelling."""
        self.x[k].copy_(self.relabel(k, x))

    def relabel(self, k, a):
        """N x D array in problem k's original labelling -> its stored labelling."""
        a = torch.as_tensor(a).to(device=self.device, dtype=torch.float64).contiguous()
        return a if self.perm[k] is None else mds_permute_rows(a, self.perm[k], False)

    def unlabel(self, k, a):
        """N x D array in problem k's stored labelling -> its original labelling."""
        return a.clone() if self.perm[k] is None else mds_permute_rows(a, self.perm[k], True)

    def eval(self, want_grad: bool = True, stream=None):
        _check(lib().mds_batch_eval(ctypes.byref(self.plan), 1 if want_grad else 0,
                                    _stream(stream)), "mds_batch_eval")

    def leapfrog(self, n_steps: int, cache_valid: bool = False, stream=None):
        """Leapfrog trajectories of n_steps steps for every problem at once
        (``mds_batch_leapfrog``): x[k] and p[k] move in place, grad[k] and
        loglik[k] end at the final positions; step[k] is eps."""
        _check(lib().mds_batch_leapfrog(ctypes.byref(self.plan), int(n_steps),
                                        1 if cache_valid else 0, _stream(stream)),
               "mds_batch_leapfrog")


def _autotuned_batch(problems, dtype, device, tile_waves):
    """Tilings of a batch from the batch tuner's cache (autotune.batch_plan):
    the common wave layout with the least predicted time and each problem's
    fastest row tile under it.  A problem that names its tile_rows keeps it;
    one whose (D, N bucket) has no entry keeps the library's batch default."""
    from . import autotune
    sizes = [(int(torch.as_tensor(p["y"]).shape[0]) if not isinstance(p["y"], torch.Tensor)
              else int(p["y"].shape[0]), int(p["d"])) for p in problems]
    tile_waves, rows = autotune.batch_plan(sizes, dtype, device, tile_waves=tile_waves)
    out = []
    for p, br in zip(problems, rows):
        q = dict(p)
        if br and "tile_rows" not in p:
            q["tile_rows"] = br
        out.append(q)
    return out, tile_waves


class HeldOutPairs:
    """The held-out pairs of a cross-validation fold on the device and the
    log pointwise predictive density over posterior draws.

    y        N x N dissimilarities (the raw values; NaN = missing)
    heldout  N x N, non-zero marks a held-out pair (read below the diagonal)
    mask     optional N x N, non-zero marks a missing pair

    ``add_draw(x, sigma)`` folds one posterior draw (x in the original
    labelling, N x D) into every pair's running average; ``lpd()`` returns the
    sum over pairs of ln(average density) as a device scalar.
    """

    def __init__(self, y, heldout, mask=None, device="cuda", stream=None):
        dev = torch.device(device)
        y = torch.as_tensor(y)
        src = y.to(device=dev, dtype=torch.float64 if y.dtype == torch.float64 else
                   torch.float32).contiguous()
        h = (torch.as_tensor(heldout) != 0).to(device=dev, dtype=torch.uint8).contiguous()
        m = None
        if mask is not None:
            m = (torch.as_tensor(mask) != 0).to(device=dev, dtype=torch.uint8).contiguous()
        n = src.shape[0]
        if src.dim() != 2 or src.shape[1] != n or h.shape != src.shape or \
                (m is not None and m.shape != src.shape):
            raise ValueError("y, heldout and mask must be N x N")
        nb = ctypes.c_size_t()
        _check(lib().mds_heldout_workspace_bytes(n, ctypes.byref(nb)), "mds_heldout_workspace_bytes")
        ws = alloc_workspace(nb.value, dev)
        cnt = torch.zeros((), dtype=torch.int64, device=dev)
        args = (_ptr(src), _dtype_code(src.dtype), _ld(src), _ptr(m), _ld(m) if m is not None else 0,
                _ptr(h), _ld(h), n)
        _check(lib().mds_heldout_count(*args, _ptr(cnt), _ptr(ws), ws.numel(),
                                       _stream(stream, src, h, m, cnt, ws)),
               "mds_heldout_count")
        self.m = int(cnt.item())
        k = max(self.m, 1)
        self.pi = torch.empty(k, dtype=torch.int32, device=dev)
        self.pj = torch.empty(k, dtype=torch.int32, device=dev)
        self.py = torch.empty(k, dtype=torch.float64, device=dev)
        _check(lib().mds_heldout_fill(*args, _ptr(ws), ws.numel(), self.m, _ptr(self.pi),
                                      _ptr(self.pj), _ptr(self.py),
                                      _stream(stream, src, h, m, ws, self.pi, self.pj, self.py)),
               "mds_heldout_fill")
        self.acc = torch.empty(2 * k, dtype=torch.float64, device=dev)
        self.draws = 0
        self.n, self.device = n, dev

    def add_draw(self, x, sigma, stream=None):
        x = torch.as_tensor(x).to(device=self.device, dtype=torch.float64)
        _check_mat(x, "x")
        if x.shape[0] != self.n:
            raise ValueError(f"x has {x.shape[0]} rows, the pairs index {self.n}")
        sig = _dev_scalar(sigma, self.device)
        _check(lib().mds_lpd_accumulate(self.m, _ptr(self.pi), _ptr(self.pj), _ptr(self.py),
                                        x.shape[1], _ptr(x), _ld(x), _ptr(sig), _ptr(self.acc),
                                        1 if self.draws == 0 else 0,
                                        _stream(stream, x, sig, self.pi, self.pj, self.py,
                                                self.acc)),
               "mds_lpd_accumulate")
        self.draws += 1

    def add_draws(self, xs, sigmas, stream=None):
        """Several posterior draws in one pass: xs is S x N x D (each draw
        contiguous), sigmas S values.  The same result, bit for bit, as S
        add_draw calls in order, with the per-pair state read and written
        once."""
        xs = torch.as_tensor(xs).to(device=self.device, dtype=torch.float64)
        if xs.dim() != 3 or xs.shape[1] != self.n:
            raise ValueError(f"xs must be S x {self.n} x D, got {tuple(xs.shape)}")
        xs = xs.contiguous()
        sig = torch.as_tensor(sigmas, dtype=torch.float64).to(self.device).reshape(-1).contiguous()
        if sig.numel() != xs.shape[0]:
            raise ValueError("one sigma per draw")
        s_draws, _, d = xs.shape
        if s_draws == 0:
            return
        _check(lib().mds_lpd_accumulate_draws(self.m, _ptr(self.pi), _ptr(self.pj),
                                              _ptr(self.py), d, _ptr(xs), d, self.n * d,
                                              _ptr(sig), s_draws, _ptr(self.acc),
                                              1 if self.draws == 0 else 0,
                                              _stream(stream, xs, sig, self.pi, self.pj,
                                                      self.py, self.acc)),
               "mds_lpd_accumulate_draws")
        self.draws += s_draws

    def lpd(self, stream=None) -> torch.Tensor:
        if self.draws == 0:
            raise ValueError("no posterior draw added")
        out = torch.empty((), dtype=torch.float64, device=self.device)
        if getattr(self, "_fin_ws", None) is None:
            nb = ctypes.c_size_t()
            _check(lib().mds_lpd_workspace_bytes(self.m, ctypes.byref(nb)),
                   "mds_lpd_workspace_bytes")
            self._fin_ws = alloc_workspace(nb.value, self.device)
        _check(lib().mds_lpd_finalize(self.m, _ptr(self.acc), self.draws, _ptr(self._fin_ws),
                                      self._fin_ws.numel(), _ptr(out),
                                      _stream(stream, self.acc, self._fin_ws, out)),
               "mds_lpd_finalize")
        return out

