"""GPU: log pointwise predictive density of held-out pairs (the
model-selection part of Section 2) -- pair compaction and the average of the
truncated-normal densities over posterior draws -- against the oracle."""
import numpy as np
import pytest
import torch

import oracle
from paper_1905_04582_amd import api, synth

pytestmark = pytest.mark.gpu

DEV = "cuda"


def _log(msg):
    print(msg, flush=True)


def _case(n, d, sigma, seed, held=0.1, missing=0.1, draws=4, nan_frac=0.0):
    pr = synth.make_problem(n, d, sigma, seed=seed, missing=missing)
    rng = np.random.Generator(np.random.PCG64(seed + 7))
    heldout = synth.symmetric_mask(n, held, rng)
    if heldout is None:
        heldout = np.zeros((n, n), dtype=np.uint8)
    y = pr.y.copy()
    if nan_frac > 0:
        bad = np.tril(rng.random((n, n)) < nan_frac, -1)
        y[bad] = np.nan
        y.T[bad] = np.nan
    xs = pr.x_true[None] + 0.05 * rng.standard_normal((draws, n, d))
    sig = sigma * rng.uniform(0.8, 1.25, draws)
    return y, heldout, pr.mask, xs, sig


def _pairs_ref(y, heldout, mask):
    n = y.shape[0]
    ii, jj = np.tril_indices(n, -1)          # row-major order of i > j
    keep = (heldout[ii, jj] != 0) & ~np.isnan(y[ii, jj])
    if mask is not None:
        keep &= mask[ii, jj] == 0
    return ii[keep], jj[keep], y[ii[keep], jj[keep]]


def _run(y, heldout, mask, xs, sig, ydtype=np.float64):
    H = api.HeldOutPairs(torch.as_tensor(y.astype(ydtype)), heldout, mask)
    for s in range(xs.shape[0]):
        H.add_draw(xs[s], float(sig[s]))
    return H, H.lpd().item()


@pytest.mark.parametrize("n,d,ydtype,nan_frac", [(300, 2, np.float64, 0.0),
                                                 (517, 3, np.float32, 0.0),
                                                 (700, 6, np.float64, 0.02),
                                                 (257, 1, np.float32, 0.02)])
def test_lpd_matches_oracle(n, d, ydtype, nan_frac):
    _log(f"lpd n={n} d={d} y={np.dtype(ydtype).name} nan={nan_frac}")
    y, heldout, mask, xs, sig = _case(n, d, 0.5, seed=n, nan_frac=nan_frac)
    yq = y.astype(ydtype).astype(np.float64)   # the values the device reads
    H, got = _run(y, heldout, mask, xs, sig, ydtype)
    ref, m = oracle.lpd(xs, sig, yq, heldout, mask)
    pi, pj, py = _pairs_ref(yq, heldout, mask)
    assert H.m == m == pi.size
    assert np.array_equal(H.pi.cpu().numpy()[:m], pi)
    assert np.array_equal(H.pj.cpu().numpy()[:m], pj)
    assert np.array_equal(H.py.cpu().numpy()[:m], py)
    _log(f"  pairs {m}: lpd {got:.15e} oracle {ref:.15e}")
    assert abs(got - ref) <= 1e-12 * abs(ref)


def test_lpd_single_draw_and_repeats():
    y, heldout, mask, xs, sig = _case(400, 2, 0.3, seed=41, draws=3)
    _, one = _run(y, heldout, mask, xs[:1], sig[:1])
    ref1, _ = oracle.lpd(xs[0], sig[0], y, heldout, mask)
    assert abs(one - ref1) <= 1e-12 * abs(ref1)
    # repeating every draw leaves the average, and so the lpd, unchanged
    _, a = _run(y, heldout, mask, xs, sig)
    _, b = _run(y, heldout, mask, np.concatenate([xs, xs]), np.concatenate([sig, sig]))
    assert abs(a - b) <= 1e-12 * abs(a)


def test_lpd_strided_x_and_device_sigma():
    y, heldout, mask, xs, sig = _case(333, 2, 0.5, seed=5)
    H = api.HeldOutPairs(torch.as_tensor(y), heldout, mask)
    for s in range(xs.shape[0]):
        wide = torch.zeros((333, 5), dtype=torch.float64, device=DEV)
        wide[:, 1:3] = torch.as_tensor(xs[s], device=DEV)
        H.add_draw(wide[:, 1:3], torch.tensor(float(sig[s]), dtype=torch.float64, device=DEV))
    ref, _ = oracle.lpd(xs, sig, y, heldout, mask)
    assert abs(H.lpd().item() - ref) <= 1e-12 * abs(ref)


def test_no_heldout_pairs_and_tiny_n():
    y, heldout, mask, xs, sig = _case(200, 2, 0.5, seed=9, held=0.0)
    H, got = _run(y, heldout, mask, xs, sig)
    assert H.m == 0 and got == 0.0
    y1 = np.zeros((1, 1))
    H1 = api.HeldOutPairs(torch.as_tensor(y1), np.ones((1, 1), np.uint8))
    H1.add_draw(np.zeros((1, 2)), 1.0)
    assert H1.m == 0 and H1.lpd().item() == 0.0
    # every pair held out, no mask
    y2, _, _, xs2, sig2 = _case(64, 2, 0.5, seed=10, missing=0.0)
    all_h = np.ones((64, 64), np.uint8)
    H2, got2 = _run(y2, all_h, None, xs2, sig2)
    ref2, m2 = oracle.lpd(xs2, sig2, y2, all_h)
    assert H2.m == m2 == 64 * 63 // 2
    assert abs(got2 - ref2) <= 1e-12 * abs(ref2)


def test_fill_respects_capacity():
    y, heldout, mask, _, _ = _case(300, 2, 0.5, seed=3)
    pi, pj, py = _pairs_ref(y, heldout, mask)
    src = torch.as_tensor(y, device=DEV)
    h = torch.as_tensor(heldout, device=DEV)
    mk = torch.as_tensor(mask, device=DEV)
    nb = api.ctypes.c_size_t()
    L = api.lib()
    assert L.mds_heldout_workspace_bytes(300, api.ctypes.byref(nb)) == 0
    ws = api.alloc_workspace(nb.value, torch.device(DEV))
    cnt = torch.zeros((), dtype=torch.int64, device=DEV)
    args = (api._ptr(src), api.MDS_F64, 300, api._ptr(mk), 300, api._ptr(h), 300, 300)
    assert L.mds_heldout_count(*args, api._ptr(cnt), api._ptr(ws), ws.numel(), None) == 0
    assert cnt.item() == pi.size
    cap = pi.size // 3
    opi = torch.full((pi.size,), -1, dtype=torch.int32, device=DEV)
    opj = torch.full((pi.size,), -1, dtype=torch.int32, device=DEV)
    opy = torch.full((pi.size,), -1.0, dtype=torch.float64, device=DEV)
    assert L.mds_heldout_fill(*args, api._ptr(ws), ws.numel(), cap, api._ptr(opi), api._ptr(opj),
                              api._ptr(opy), None) == 0
    torch.cuda.synchronize()
    assert np.array_equal(opi.cpu().numpy()[:cap], pi[:cap])
    assert np.array_equal(opj.cpu().numpy()[:cap], pj[:cap])
    assert np.array_equal(opy.cpu().numpy()[:cap], py[:cap])
    assert (opi.cpu().numpy()[cap:] == -1).all() and (opy.cpu().numpy()[cap:] == -1.0).all()


def test_lpd_paper_scale():
    """N = 5392 locations, D = 2, 10% of the pairs held out, 15% missing,
    four posterior draws."""
    _log("lpd paper scale n=5392")
    y, heldout, mask, xs, sig = _case(5392, 2, 0.3, seed=5392, missing=0.15)
    H, got = _run(y, heldout, mask, xs, sig)
    ref, m = oracle.lpd(xs, sig, y, heldout, mask)
    _log(f"  pairs {m}: lpd {got:.15e} oracle {ref:.15e}")
    assert H.m == m
    assert abs(got - ref) <= 1e-12 * abs(ref)


@pytest.mark.parametrize("n,d,draws", [(300, 2, 5), (1500, 3, 7), (257, 6, 3)])
def test_many_draws_per_pass_equal_single_draws_bitwise(n, d, draws):
    # one pass over S draws equals S single-draw passes bit for bit, also
    # after a first single draw (continuing sums), and matches the oracle
    _log(f"lpd draws per pass: n={n} d={d} S={draws}")
    y, heldout, mask, xs, sig = _case(n, d, 0.4, seed=n + 1, draws=draws, nan_frac=0.01)
    H1, got1 = _run(y, heldout, mask, xs, sig)
    H2 = api.HeldOutPairs(torch.as_tensor(y), heldout, mask)
    H2.add_draws(xs, sig)
    H3 = api.HeldOutPairs(torch.as_tensor(y), heldout, mask)
    H3.add_draw(xs[0], float(sig[0]))
    H3.add_draws(xs[1:], sig[1:])
    H3.add_draws(xs[:0], sig[:0])                      # no draws: nothing changes
    assert H2.draws == H3.draws == draws
    k = 2 * H1.m
    a1 = H1.acc.cpu().numpy()[:k]
    assert np.array_equal(a1, H2.acc.cpu().numpy()[:k])
    assert np.array_equal(a1, H3.acc.cpu().numpy()[:k])
    got2, got3 = H2.lpd().item(), H3.lpd().item()
    assert got1 == got2 == got3
    ref, _ = oracle.lpd(xs, sig, y, heldout, mask)
    _log(f"  pairs {H1.m}: lpd {got2:.15e} oracle {ref:.15e}")
    assert abs(got2 - ref) <= 1e-12 * abs(ref)


def test_draws_on_a_caller_stream_with_host_inputs():
    # draws passed as host arrays and Python floats (temporaries the binding
    # converts) on a stream other than torch's current one: the binding keeps
    # them alive for that stream, and the result equals the same draws made
    # on the current stream, bit for bit
    p = synth.make_problem(300, 2, 0.6, seed=81, missing=0.1)
    held = synth.symmetric_mask(300, 0.2, np.random.default_rng(82))
    xs = [p.x + 0.02 * k for k in range(4)]
    H0 = api.HeldOutPairs(p.y, held, p.mask, DEV)
    for k, x in enumerate(xs):
        H0.add_draw(x, p.sigma * (1 + 0.1 * k))
    ref = H0.lpd().item()
    side = torch.cuda.Stream()
    H1 = api.HeldOutPairs(p.y, held, p.mask, DEV)
    side.wait_stream(torch.cuda.current_stream())
    for k, x in enumerate(xs):
        H1.add_draw(x, p.sigma * (1 + 0.1 * k), stream=side)
        torch.empty(1 << 20, dtype=torch.float64, device=DEV).fill_(7.0)   # churn the allocator
    out = H1.lpd(stream=side)
    side.synchronize()
    assert out.item() == ref
