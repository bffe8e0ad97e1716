"""Batched form: many independent problems of uneven N and D in one
persistent launch.  Every problem must equal, bit for bit, its own
single-problem call with the same tiling, and the oracle to 1e-12 (FP64)."""
import numpy as np
import pytest
import torch

import oracle
from paper_1905_04582_amd import api, synth

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _mixed_specs(seed, count=10):
    rng = np.random.default_rng(seed)
    dims = [1, 2, 3, 4, 6, 8, 2, 5, 7, 2, 4, 6]
    out = []
    for k in range(count):
        n = int(rng.integers(2, 900)) if k else 1
        out.append(dict(n=n, d=dims[k % len(dims)], sigma=float(rng.uniform(0.2, 1.0)),
                        missing=0.1, seed=9000 + k))
    return out


def _build(specs, dtype, tile_rows=0):
    probs = [synth.make_problem(**s) for s in specs]
    B = api.MDSBatch([dict(y=p.y.astype(np.float32) if dtype == torch.float32 else p.y, d=p.d,
                           mask=p.mask, tile_rows=tile_rows) for p in probs], dtype, DEV)
    for k, p in enumerate(probs):
        B.set_x(k, p.x)
        B.sigma[k] = p.sigma
    return probs, B


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_batch_equals_single_calls_bitwise(dtype):
    probs, B = _build(_mixed_specs(1), dtype)
    B.eval()
    torch.cuda.synchronize()
    for k, p in enumerate(probs):
        P = api.MDSProblem(p.y.astype(np.float32) if dtype == torch.float32 else p.y, p.d,
                           p.mask, dtype, DEV, *B.tiles[k])
        g, L, ds = P.gradient(B.x[k], p.sigma)
        torch.cuda.synchronize()
        assert torch.equal(g, B.grad[k]), k
        assert L.item() == B.loglik[k].item() and ds.item() == B.dsigma[k].item(), k


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_relabelled_batch_equals_single_calls_bitwise(dtype):
    # problems stored in the spatial order of their locations: every problem
    # equals its relabelled single-problem call, and the oracle in the
    # original labelling
    specs = _mixed_specs(11, 8)
    probs = [synth.make_problem(**sp) for sp in specs]
    yv = [p.y.astype(np.float32) if dtype == torch.float32 else p.y for p in probs]
    B = api.MDSBatch([dict(y=y, d=p.d, mask=p.mask, order=p.x) for y, p in zip(yv, probs)],
                     dtype, DEV)
    for k, p in enumerate(probs):
        B.set_x(k, p.x)
        B.sigma[k] = p.sigma
    B.eval()
    torch.cuda.synchronize()
    for k, p in enumerate(probs):
        P = api.MDSProblem(yv[k], p.d, p.mask, dtype, DEV, *B.tiles[k], order=p.x)
        g, L, _ = P.gradient(P.relabel(p.x), p.sigma)
        torch.cuda.synchronize()
        assert torch.equal(B.perm[k], P.perm), k
        assert torch.equal(g, B.grad[k]) and L.item() == B.loglik[k].item(), k
        if dtype == torch.float64 and p.n > 1:
            ref = oracle.evaluate(p.x, p.y, p.sigma, p.mask)
            got = B.unlabel(k, B.grad[k]).cpu().numpy()
            assert np.all(np.max(np.abs(got - ref.grad), axis=1) <= 1e-12 * ref.condrow), k


def test_batch_fp64_vs_oracle_and_repeat():
    probs, B = _build(_mixed_specs(2, 12), torch.float64)
    B.eval()
    torch.cuda.synchronize()
    first = [g.clone() for g in B.grad]
    for k, p in enumerate(probs):
        ref = oracle.evaluate(p.x, p.y, p.sigma, p.mask)
        L = B.loglik[k].item()
        assert abs(L - ref.loglik) <= 1e-12 * max(abs(ref.loglik), 1e-300) + 1e-300, k
        rowerr = np.max(np.abs(B.grad[k].cpu().numpy() - ref.grad), axis=1) if p.n else 0
        assert np.all(rowerr <= 1e-12 * ref.condrow + 1e-300), k
        assert abs(B.dlogsigma[k].item() - p.sigma * ref.dsigma) <= \
            1e-12 * p.sigma * ref.abs_dsigma + 1e-300
    # the tile cursor rewinds: a second evaluation is identical
    B.eval()
    torch.cuda.synchronize()
    for k in range(len(probs)):
        assert torch.equal(first[k], B.grad[k])
    # log-likelihood only
    L1 = B.loglik.clone()
    B.loglik.zero_()
    B.eval(want_grad=False)
    torch.cuda.synchronize()
    assert torch.equal(L1, B.loglik)


def test_batch_graph_capture():
    probs, B = _build(_mixed_specs(3, 8), torch.float32)
    B.eval()
    torch.cuda.synchronize()
    ref = [g.clone() for g in B.grad]
    refL = B.loglik.clone()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        B.eval()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    G = torch.cuda.CUDAGraph()
    with torch.cuda.graph(G):
        B.eval()
    for rep in range(3):
        for g in B.grad:
            g.zero_()
        G.replay()
        torch.cuda.synchronize()
        assert all(torch.equal(a, b) for a, b in zip(ref, B.grad)), rep
        assert torch.equal(refL, B.loglik)
        _ = B.x[0].sum().item()


def test_batched_workload_64_problems():
    # 64 problems, N ~ U[500, 8000], D in {2, 4, 6}, sigma ~ U(0.2, 1), FP32 Y,
    # 10% missing: bitwise equal to single calls; a few against the oracle
    specs = synth.batch_specs(64, seed=64)
    probs, B = _build(specs, torch.float32)
    B.eval()
    torch.cuda.synchronize()
    for k in (0, 17, 41, 63):
        p = probs[k]
        P = api.MDSProblem(p.y.astype(np.float32), p.d, p.mask, torch.float32, DEV, *B.tiles[k])
        g, L, _ = P.gradient(B.x[k], p.sigma)
        torch.cuda.synchronize()
        assert torch.equal(g, B.grad[k]) and L.item() == B.loglik[k].item()
    small = min(range(64), key=lambda k: probs[k].n)
    p = probs[small]
    ref = oracle.evaluate(p.x, p.y.astype(np.float32).astype(np.float64), p.sigma, p.mask)
    assert abs(B.loglik[small].item() - ref.loglik) <= 1e-5 * abs(ref.loglik)
    rows = np.arange(0, p.n, max(1, p.n // 20))
    g, a, b = oracle.grad_rows(p.x, p.y.astype(np.float32).astype(np.float64), p.sigma, rows,
                               p.mask)
    err = np.max(np.abs(B.grad[small].cpu().numpy()[rows] - g), axis=1) / b
    assert err.max() < 1e-5


# ------------------------------------------------------------ leapfrog ----

def _start(B, probs, seed):
    rng = np.random.default_rng(seed)
    moms = []
    for k, p in enumerate(probs):
        m = rng.standard_normal((p.n, p.d))
        B.p[k].copy_(torch.as_tensor(m))
        B.step[k] = float(rng.uniform(5e-4, 2e-3))
        moms.append(m)
    return moms


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_batch_leapfrog_equals_single_calls_bitwise(dtype):
    probs, B = _build(_mixed_specs(5, 9), dtype)
    moms = _start(B, probs, 5)
    B.leapfrog(7)
    B.leapfrog(4, cache_valid=True)
    torch.cuda.synchronize()
    for k, p in enumerate(probs):
        P = api.MDSProblem(p.y.astype(np.float32) if dtype == torch.float32 else p.y, p.d,
                           p.mask, dtype, DEV, *B.tiles[k])
        x = torch.as_tensor(p.x, dtype=torch.float64, device=DEV).clone()
        pm = torch.as_tensor(moms[k], dtype=torch.float64, device=DEV).clone()
        g = torch.empty_like(x)
        L = torch.empty((), dtype=torch.float64, device=DEV)
        st = B.step[k].clone()
        P.leapfrog(x, pm, p.sigma, st, 7, g, L)
        P.leapfrog(x, pm, p.sigma, st, 4, g, L, cache_valid=True)
        torch.cuda.synchronize()
        assert torch.equal(x, B.x[k]) and torch.equal(pm, B.p[k]), k
        assert torch.equal(g, B.grad[k]) and L.item() == B.loglik[k].item(), k


def test_batch_leapfrog_vs_oracle():
    probs, B = _build(_mixed_specs(6, 8), torch.float64)
    moms = _start(B, probs, 6)
    B.leapfrog(20)
    torch.cuda.synchronize()
    for k, p in enumerate(probs):
        eps = B.step[k].item()
        ref = oracle.leapfrog(p.x, moms[k], p.y, p.sigma, eps=eps, n_steps=20, mask=p.mask)
        gx, gp = B.x[k].cpu().numpy(), B.p[k].cpu().numpy()
        if p.n == 0:
            continue
        ev = oracle.evaluate(ref.x, p.y, p.sigma, p.mask)
        ptol = 1e-12 * eps * 21 * max(np.max(ev.condrow), 1e-300) + 1e-300
        assert np.abs(gx - ref.x).max() <= 1e-12 * max(np.abs(ref.x).max(), 1e-300), k
        assert np.abs(gp - ref.p).max() <= ptol, k
        assert abs(B.loglik[k].item() - ref.loglik_end) <= \
            1e-11 * max(abs(ref.loglik_end), 1e-300) + 1e-300, k


def test_batch_leapfrog_graph_replays():
    # 20-step trajectories of the whole batch captured once, replayed; each
    # replay continues from the last (cached gradient) and equals the eager
    # batch run step for step
    probs, B = _build(_mixed_specs(7, 8), torch.float32)
    _start(B, probs, 7)
    B.leapfrog(0)                                  # gradient at the start
    probs2, E = _build(_mixed_specs(7, 8), torch.float32)
    _start(E, probs2, 7)
    E.leapfrog(0)
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    G = torch.cuda.CUDAGraph()
    x0 = [x.clone() for x in B.x]
    p0 = [p.clone() for p in B.p]
    with torch.cuda.stream(side):
        B.leapfrog(20, cache_valid=True)           # warm the capture stream
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    for k in range(B.count):                       # back to the start
        B.x[k].copy_(x0[k])
        B.p[k].copy_(p0[k])
    B.leapfrog(0)
    torch.cuda.synchronize()
    with torch.cuda.graph(G):
        B.leapfrog(20, cache_valid=True)
    for rep in range(3):
        G.replay()
        E.leapfrog(20, cache_valid=True)
        torch.cuda.synchronize()
        for k in range(B.count):
            assert torch.equal(B.x[k], E.x[k]) and torch.equal(B.p[k], E.p[k]), (rep, k)
            assert torch.equal(B.grad[k], E.grad[k]), (rep, k)
        assert torch.equal(B.loglik, E.loglik), rep
