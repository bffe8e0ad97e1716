"""GPU: mds_gradient_noalloc (the fused evaluation with its partial sums in
the library's static device scratch, no workspace argument) through the C ABI
against mds_gradient with a workspace: the same kernels and tiling, so the
outputs must agree bit for bit; two calls in a row, the second on a smaller
problem (the scratch keeps the first call's contents), and the paper-scale
problem also against the oracle."""
import numpy as np
import pytest
import torch

import oracle
from paper_1905_04582_amd import api, synth

pytestmark = pytest.mark.gpu

DEV = "cuda"


def _both(P, x, sigma):
    """(with a workspace, without one) on the same problem and stream."""
    sig = torch.tensor(sigma, dtype=torch.float64, device=DEV)
    g_ws, L_ws, ds_ws = P.gradient(x, sig)
    g0 = torch.empty_like(x)
    L0 = torch.empty((), dtype=torch.float64, device=DEV)
    d0 = torch.empty((), dtype=torch.float64, device=DEV)
    api.mds_gradient_noalloc(x, P.y, sig, g0, L0, d0, tile_rows=P.tile_rows,
                             tile_waves=P.tile_waves, truncated=P.truncated)
    torch.cuda.synchronize()
    return (g_ws.cpu().numpy(), L_ws.item(), ds_ws.item()), (g0.cpu().numpy(), L0.item(), d0.item())


def _same(a, b, label):
    (ga, la, da), (gb, lb, db) = a, b
    print(f"{label}: max |grad diff| {np.max(np.abs(ga - gb)) if ga.size else 0.0:.1e}, "
          f"L {la!r} vs {lb!r}", flush=True)
    assert np.array_equal(ga, gb) and la == lb and da == db, label


def test_noalloc_matches_workspace_call_twice_second_smaller():
    # first call: the paper-scale problem (N = 5392, 11.2 MB of partials)
    p = synth.preset("paper_fp64")
    P = api.MDSProblem(p.y, p.d, p.mask, torch.float64, DEV)
    x = torch.as_tensor(p.x, device=DEV)
    ws, st = _both(P, x, p.sigma)
    _same(ws, st, "N=5392 FP64")
    ref = oracle.evaluate(p.x, p.y, p.sigma, p.mask)
    assert abs(st[1] - ref.loglik) <= 1e-12 * abs(ref.loglik)
    assert np.all(np.max(np.abs(st[0] - ref.grad), axis=1) <= 1e-12 * ref.condrow)
    del P
    # second call, smaller: FP32 form, D = 3, N = 700 (the scratch still holds
    # the first call's partial sums)
    q = synth.make_problem(700, 3, 0.6, seed=71, missing=0.1)
    Q = api.MDSProblem(q.y.astype(np.float32), q.d, q.mask, torch.float32, DEV)
    xq = torch.as_tensor(q.x, device=DEV)
    ws2, st2 = _both(Q, xq, q.sigma)
    _same(ws2, st2, "N=700 D=3 FP32")
    # and a third, smaller again, with the untruncated model and row waves
    r = synth.make_problem(300, 2, 0.8, seed=72)
    R = api.MDSProblem(r.y, r.d, None, torch.float64, DEV, 64, api.tile_waves(1, 4),
                       truncated=False)
    _same(*_both(R, torch.as_tensor(r.x, device=DEV), r.sigma), "N=300 untruncated row waves")


def test_noalloc_rejects_a_problem_beyond_the_scratch():
    n = 20000
    x = torch.zeros((n, 2), dtype=torch.float64, device=DEV)
    y = torch.zeros((n, api.padded_ld(n)), dtype=torch.float64, device=DEV)[:, :n]
    sig = torch.ones((), dtype=torch.float64, device=DEV)
    g = torch.empty_like(x)
    with pytest.raises(api.MDSError) as e:
        api.mds_gradient_noalloc(x, y, sig, g)
    assert e.value.status == api.MDS_ERR_WORKSPACE_TOO_SMALL
