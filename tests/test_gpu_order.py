"""GPU: spatial relabelling (mds_spatial_order, mds_permute_rows, relabelled
mds_prepare_y) and the evaluation of relabelled problems against the oracle.

The order is integer work and must equal the numpy statement in
tests/order_ref.py exactly.  A relabelled evaluation must give the oracle's L
and dL/dsigma and, after mapping the rows back, its gradient, to the same
tolerances as the plain evaluation; at the paper-scale workload most
wavefronts of the relabelled sweep skip the truncation terms, so these cases
exercise that branch.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1905_04582_amd import api, synth
from tests import order_ref
from tests.test_gpu_parity import DEV, TOL32_LOGLIK, check64

pytestmark = pytest.mark.gpu


def _log(msg):
    print(msg, flush=True)


@pytest.mark.parametrize("d", [1, 2, 3, 6, 8])
@pytest.mark.parametrize("n", [0, 1, 7, 1000, 5392])
def test_order_matches_statement(n, d):
    rng = np.random.default_rng(1000 * d + n)
    x = rng.standard_normal((n, d)) * 3.0
    if n >= 7:
        x[3] = x[5]                  # exact ties keep index order
        x[6, 0] = np.nan             # NaN coordinates quantise to 0
    xt = torch.as_tensor(x, device=DEV)
    perm = api.mds_spatial_order(xt).cpu().numpy()
    want = order_ref.spatial_order(x)
    _log(f"order n={n} d={d}: {int(np.sum(perm != want))} mismatches")
    assert perm.tolist() == want.tolist()


def test_order_strided_x():
    rng = np.random.default_rng(5)
    xb = torch.as_tensor(rng.standard_normal((500, 5)), device=DEV)
    x = xb[:, :2]
    perm = api.mds_spatial_order(x).cpu().numpy()
    assert perm.tolist() == order_ref.spatial_order(x.cpu().numpy()).tolist()


def test_permute_rows_round_trip():
    rng = np.random.default_rng(9)
    x = rng.standard_normal((777, 3))
    xt = torch.as_tensor(x, device=DEV)
    perm = api.mds_spatial_order(xt)
    fwd = api.mds_permute_rows(xt, perm)
    back = api.mds_permute_rows(fwd, perm, inverse=True)
    p = perm.cpu().numpy()
    assert np.array_equal(fwd.cpu().numpy(), x[p])
    assert np.array_equal(back.cpu().numpy(), x)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_prepare_relabelled(dtype):
    rng = np.random.default_rng(11)
    n = 300
    y = np.abs(rng.standard_normal((n, n)))
    y = np.tril(y, -1)
    y = y + y.T
    m = np.tril(rng.random((n, n)) < 0.2, -1)
    mask = (m | m.T).astype(np.uint8)
    y[5, 9] = y[9, 5] = np.nan
    perm = torch.as_tensor(rng.permutation(n), device=DEV)
    yp, mo = api.mds_prepare_y(torch.as_tensor(y, device=DEV), dtype,
                               torch.as_tensor(mask, device=DEV), perm=perm)
    p = perm.cpu().numpy()
    want = y[p][:, p].copy()
    want[mask[p][:, p] != 0] = np.nan
    got = yp[:, :n].cpu().numpy().astype(np.float64)
    assert np.array_equal(np.isnan(got), np.isnan(want))
    ok = ~np.isnan(want)
    assert np.array_equal(got[ok], want[ok].astype(np.dtype(str(dtype).split(".")[1])))
    _, mo0 = api.mds_prepare_y(torch.as_tensor(y, device=DEV), dtype,
                               torch.as_tensor(mask, device=DEV))
    assert mo.item() == mo0.item()


def _relabelled_eval(prob, dtype):
    P = api.MDSProblem(prob.y, prob.d, prob.mask, dtype, DEV, order=prob.x)
    xi = P.relabel(prob.x)
    g, L, ds = P.gradient(xi, prob.sigma)
    L2 = P.loglik(xi, prob.sigma)
    gu = P.unlabel(g)
    torch.cuda.synchronize()
    return dict(grad=gu.cpu().numpy(), loglik=L.item(), dsigma=ds.item(),
                loglik_only=L2.item(), m_obs=int(P.m_obs.item()))


@pytest.mark.parametrize("name", ["small_fp64", "paper_fp64"])
def test_relabelled_fp64_parity(name):
    prob = synth.preset(name)
    ref = oracle.evaluate(prob.x, prob.y, prob.sigma, prob.mask)
    got = _relabelled_eval(prob, torch.float64)
    check64(got, ref, f"{name} relabelled")


@pytest.mark.parametrize("name", ["paper_fp32_d2", "paper_fp32_d6_tight"])
def test_relabelled_fp32_loglik(name):
    prob = synth.preset(name)
    y32 = prob.y.astype(np.float32).astype(np.float64)
    ref = oracle.evaluate(prob.x, y32, prob.sigma, prob.mask)
    got = _relabelled_eval(prob, torch.float32)
    rel = abs(got["loglik"] - ref.loglik) / abs(ref.loglik)
    rowerr = np.max(np.abs(got["grad"] - ref.grad), axis=1)
    _log(f"{name} relabelled FP32: loglik rel {rel:.2e}, grad row err/B_i "
         f"{np.max(rowerr / ref.condrow):.2e}")
    assert got["m_obs"] == ref.m_obs
    assert rel <= TOL32_LOGLIK


def test_relabelled_leapfrog_matches_plain():
    """A trajectory in the relabelled frame, mapped back, equals the plain one
    to the FP64 tolerance of the positions (same arithmetic up to the skip)."""
    prob = synth.preset("small_fp64")
    n, d = prob.x.shape
    mom = np.random.default_rng(3).standard_normal((n, d))
    outs = []
    for order in (None, prob.x):
        P = api.MDSProblem(prob.y, d, prob.mask, torch.float64, DEV, order=order)
        x = P.relabel(prob.x)
        p = P.relabel(mom)
        g = torch.empty_like(x)
        L = torch.empty((), dtype=torch.float64, device=DEV)
        P.leapfrog(x, p, prob.sigma, 1e-3, 20, g, L)
        outs.append((P.unlabel(x).cpu().numpy(), P.unlabel(p).cpu().numpy(), L.item()))
    (x0, p0, l0), (x1, p1, l1) = outs
    assert np.max(np.abs(x0 - x1)) <= 1e-12 * np.max(np.abs(x0))
    assert np.max(np.abs(p0 - p1)) <= 1e-9 * np.max(np.abs(p0))
    assert abs(l0 - l1) <= 1e-12 * abs(l0)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_check_symmetric(dtype):
    rng = np.random.default_rng(12)
    n = 257
    y = np.abs(rng.standard_normal((n, n)))
    y = np.tril(y, -1)
    y = y + y.T
    y[3, 7] = y[7, 3] = np.nan                      # a missing pair on both sides: fine
    yt = torch.as_tensor(y, dtype=dtype, device=DEV)
    assert api.mds_check_symmetric(yt) == 0
    yt[10, 2] += 1.0
    yt[100, 200] = float("nan")                    # missing on one side only
    assert api.mds_check_symmetric(yt) == 2
    # an asymmetric mask shows up in the prepared matrix
    mask = np.zeros((n, n), np.uint8)
    mask[5, 1] = 1
    with pytest.raises(api.MDSError) as e:
        api.MDSProblem(y, 2, mask, dtype, DEV, check_symmetric=True)
    assert e.value.status == api.MDS_ERR_NOT_SYMMETRIC
    api.MDSProblem(y, 2, None, dtype, DEV, check_symmetric=True)
