"""GPU: the fused evaluation at the largest sizes of the N sweep (the paper's
scaling study over randomly sampled 2-D Gaussian points), with Y drawn in
device memory: sampled gradient rows (Eq. 9) against the row oracle, the
zero sum of the gradient rows, and L in two labellings."""
import numpy as np
import pytest
import torch

import oracle
from paper_1905_04582_amd import api, synth

pytestmark = pytest.mark.gpu

DEV = "cuda"
TOL64 = 1e-12


def _log(msg):
    print(msg, flush=True)


def _eval(P, x, sigma):
    xr = P.relabel(torch.as_tensor(x, device=DEV))
    g, L, ds = P.gradient(xr, sigma)
    torch.cuda.synchronize()
    return P.unlabel(g).cpu().numpy(), L.item(), ds.item()


@pytest.mark.parametrize("n", [50000, 100000])
def test_large_n_sampled_rows(n):
    _log(f"N sweep parity: N={n} D=2 sigma=0.5, Y drawn on the device")
    sigma = 0.5
    x_true, x, y = synth.device_problem(n, 2, sigma, seed=n, device=DEV)
    rows = np.concatenate([np.random.default_rng(n).choice(n, 30, replace=False), [0, n - 1]])
    yrows = y[torch.as_tensor(rows, device=DEV)].cpu().numpy()
    gref, a, b = oracle.grad_rows_given(x, yrows, sigma, rows)

    P = api.MDSProblem(y, 2, None, torch.float64, DEV, order=x)
    g64, L64, ds64 = _eval(P, x, sigma)
    del P
    err = np.max(np.abs(g64[rows] - gref), axis=1)
    _log(f"  fp64 sampled rows: max err/B_i {np.max(err / b):.2e}")
    assert np.all(err <= TOL64 * b)
    # every pair enters two rows with opposite signs: the rows sum to zero
    # up to the rounding of the N row sums, each bounded like a sampled row
    colsum = np.abs(g64.sum(axis=0)).max()
    _log(f"  fp64 |sum of rows| {colsum:.2e} against N median(B_i) {n * np.median(b):.2e}")
    assert colsum <= TOL64 * n * np.median(b)
    assert np.isfinite(L64) and np.isfinite(ds64)

    if n <= 50000:
        # the original labelling (no relabelling): same L up to rounding
        Q = api.MDSProblem(y, 2, None, torch.float64, DEV)
        _, Lq, _ = _eval(Q, x, sigma)
        del Q
        _log(f"  fp64 L relabelled {L64:.15e} original {Lq:.15e}")
        assert abs(L64 - Lq) <= TOL64 * abs(Lq)

    P32 = api.MDSProblem(y, 2, None, torch.float32, DEV, order=x)
    del y
    torch.cuda.empty_cache()
    g32, L32, _ = _eval(P32, x, sigma)
    yr32 = yrows.astype(np.float32).astype(np.float64)
    g32ref, _, b32 = oracle.grad_rows_given(x, yr32, sigma, rows)
    err32 = np.max(np.abs(g32[rows] - g32ref), axis=1) / b32
    rel = abs(L32 - L64) / abs(L64)
    _log(f"  fp32 sampled rows: max err/B_i {err32.max():.2e}; L rel diff vs FP64 {rel:.2e}")
    assert err32.max() <= 2.0 ** -17      # the FP32 form's stated row bound
    # FP64 L of FP64 Y against FP32 of FP32-rounded Y: the rounding of Y
    # itself moves L by well under the FP32 bound
    assert rel <= 1e-5
