"""GPU: the HMC transition (Section 2.3) -- momentum draw, Metropolis test,
restore on rejection, graph-captured chains -- against the oracle's
transition with the same Philox draws."""
import math

import numpy as np
import pytest
import torch

import oracle
from paper_1905_04582_amd import api, graphs, synth

pytestmark = pytest.mark.gpu

DEV = "cuda"
f64 = dict(dtype=torch.float64, device=DEV)


def _log(msg):
    print(msg, flush=True)


def _counter(v):
    # an int64 device scalar holding the uint64 transition index v
    if v >= 1 << 63:
        v -= 1 << 64
    return torch.tensor([v], dtype=torch.int64, device=DEV)


@pytest.mark.parametrize("seed,it", [(0, 0), (12345, 7), ((1 << 40) + 5, (1 << 33) + 7),
                                     ((1 << 64) - 1, (1 << 64) - 2)])
def test_momentum_matches_oracle(seed, it):
    n, d = 1001, 3
    im = np.random.default_rng(1).uniform(0.25, 4.0, (n, d))
    ref = oracle.momentum(n, d, seed, it, inv_mass=im)
    got = api.mds_hmc_momentum(n, d, seed, _counter(it),
                               inv_mass=torch.as_tensor(im, **f64)).cpu().numpy()
    err = np.abs(got - ref).max()
    _log(f"momentum seed={seed} it={it}: max |dp| {err:.2e}")
    assert err <= 1e-13


def _gpu_chain(P, x, sigma, eps, n_steps, seed, its, prior=None):
    """Transitions its[0], its[1], ... from x, all in the problem's labelling."""
    x = torch.as_tensor(x, **f64).clone()
    p = torch.empty_like(x)
    g = torch.empty_like(x)
    L = torch.empty((), **f64)
    it = _counter(its[0])
    stats = torch.empty(4, **f64)
    acc = torch.zeros(1, dtype=torch.int64, device=DEV)
    out = []
    for k in range(len(its)):
        P.hmc_step(x, p, sigma, eps, n_steps, seed, it, g, L, cache_valid=k > 0, prior=prior,
                   stats=stats, accepted_total=acc)
        out.append(dict(x=x.cpu().numpy(), g=g.cpu().numpy(), L=L.item(),
                        stats=stats.cpu().numpy().copy()))
    assert it.item() == its[0] + len(its) and acc.item() == sum(int(o["stats"][3]) for o in out)
    return out


def _labelled(P, prob):
    """The problem as the device holds it: the momentum draws follow the
    problem's labelling, so the oracle runs on the relabelled inputs."""
    if P.perm is None:
        return prob.x, prob.y, prob.mask
    q = P.perm.cpu().numpy()
    mask = None if prob.mask is None else prob.mask[q][:, q]
    return prob.x[q], prob.y[q][:, q], mask


@pytest.mark.parametrize("ordered", [False, True])
def test_chain_matches_oracle(ordered):
    pr = synth.preset("small_fp64")
    P = api.MDSProblem(pr.y, pr.d, pr.mask, torch.float64, DEV, order=pr.x if ordered else None)
    x, y, mask = _labelled(P, pr)
    seed, its, eps, steps = 77, list(range(40, 46)), 0.02, 10
    got = _gpu_chain(P, x, pr.sigma, eps, steps, seed, its)
    n_acc = 0
    for k, it in enumerate(its):
        ref = oracle.hmc_step(x, y, pr.sigma, eps, steps, seed, it, mask=mask)
        h0, h1, lu, acc = got[k]["stats"]
        margin = abs(ref.log_u - (ref.energy_start - ref.energy_end))
        _log(f"transition {it}: accepted {ref.accepted}/{bool(acc)} dH {h1 - h0:.3e} "
             f"margin {margin:.2e}")
        assert abs(h0 - ref.energy_start) <= 1e-11 * abs(ref.energy_start)
        assert abs(h1 - ref.energy_end) <= 1e-11 * abs(ref.energy_end)
        assert abs(lu - ref.log_u) <= 1e-15 * max(1.0, abs(ref.log_u))
        if margin < 1e-8 * abs(ref.energy_start):
            pytest.skip("a Metropolis test within rounding of its threshold")
        assert bool(acc) == ref.accepted
        n_acc += ref.accepted
        assert np.abs(got[k]["x"] - ref.x).max() <= 1e-12 * np.abs(ref.x).max()
        assert abs(got[k]["L"] - ref.loglik) <= 1e-11 * abs(ref.loglik)
        ev = oracle.evaluate(ref.x, y, pr.sigma, mask)
        assert np.all(np.max(np.abs(got[k]["g"] - ref.grad), axis=1) <= 1e-10 * ev.condrow)
        x = ref.x
    _log(f"accepted {n_acc} of {len(its)}")


def test_rejection_restores_state_bitwise():
    p = synth.preset("small_fp64")
    P = api.MDSProblem(p.y, p.d, p.mask, torch.float64, DEV)
    x = torch.as_tensor(p.x, **f64).clone()
    g = torch.empty_like(x)
    L = torch.empty((), **f64)
    P.leapfrog(x, torch.zeros_like(x), p.sigma, 1.0, 0, g, L, prior=0.5)
    x0, g0, L0 = x.clone(), g.clone(), L.clone()
    stats = torch.empty(4, **f64)
    it = _counter(3)
    P.hmc_step(x, torch.empty_like(x), p.sigma, 5.0, 8, 1, it, g, L, cache_valid=True,
               prior=0.5, stats=stats)
    s = stats.cpu().numpy()
    _log(f"exploding step: H {s[0]:.3e} -> {s[1]:.3e}, accepted {s[3]}")
    assert s[3] == 0.0 and it.item() == 4
    assert torch.equal(x, x0) and torch.equal(g, g0) and torch.equal(L, L0)


def test_chain_untruncated_matches_oracle():
    """Transitions of the model without truncation (the MDS_UNTRUNCATED flag
    of mds_hmc_step) against the oracle's, in the spatial labelling."""
    pr = synth.preset("small_fp64", missing=0.1)
    P = api.MDSProblem(pr.y, pr.d, pr.mask, torch.float64, DEV, order=pr.x, truncated=False)
    x, y, mask = _labelled(P, pr)
    seed, its, eps, steps = 78, list(range(10, 14)), 0.02, 8
    got = _gpu_chain(P, x, pr.sigma, eps, steps, seed, its)
    for k, it in enumerate(its):
        ref = oracle.hmc_step(x, y, pr.sigma, eps, steps, seed, it, mask=mask, truncated=False)
        h0, h1, lu, acc = got[k]["stats"]
        margin = abs(ref.log_u - (ref.energy_start - ref.energy_end))
        _log(f"untruncated transition {it}: accepted {ref.accepted}/{bool(acc)} "
             f"margin {margin:.2e}")
        assert abs(h0 - ref.energy_start) <= 1e-11 * abs(ref.energy_start)
        assert abs(h1 - ref.energy_end) <= 1e-11 * abs(ref.energy_end)
        if margin >= 1e-8 * abs(ref.energy_start):
            assert bool(acc) == ref.accepted
            assert np.abs(got[k]["x"] - ref.x).max() <= 1e-12 * np.abs(ref.x).max()
            assert abs(got[k]["L"] - ref.loglik) <= 1e-11 * abs(ref.loglik)
        x = got[k]["x"]          # continue from the device's state


def test_chain_graph_replays_match_eager():
    pr = synth.make_problem(400, 2, 0.6, seed=9, missing=0.1)
    P = api.MDSProblem(pr.y, 2, pr.mask, torch.float64, DEV, order=pr.x)
    G = graphs.HMCChainGraph(P, P.relabel(pr.x), n_steps=6, sigma=pr.sigma, step=0.02, seed=5,
                             prior=0.1, transitions_per_graph=2, first_iteration=100)
    # the eager chain, two transitions per replay
    x = P.relabel(pr.x)
    p = torch.empty_like(x)
    g = torch.empty_like(x)
    L = torch.empty((), **f64)
    it = _counter(100)
    first = True
    for rep in range(3):
        G.run(1)
        torch.cuda.synchronize()
        for _ in range(2):
            P.hmc_step(x, p, pr.sigma, 0.02, 6, 5, it, g, L, cache_valid=not first, prior=0.1)
            first = False
        torch.cuda.synchronize()
        assert G.iteration.item() == it.item() == 100 + 2 * (rep + 1)
        assert torch.equal(G.x, x), rep
        assert torch.equal(G.grad, g) and torch.equal(G.loglik, L)


def test_chain_samples_gaussian_target():
    """All pairs missing, prior precision lambda: N(0, I/lambda) exactly; the
    GPU chain makes the oracle chain's decisions."""
    n, d, lam = 25, 2, 2.0
    y = np.ones((n, n))
    mask = np.ones((n, n), np.uint8)
    P = api.MDSProblem(y, d, mask, torch.float64, DEV)
    G = graphs.HMCChainGraph(P, np.zeros((n, d)), n_steps=4, sigma=1.0, step=0.4, seed=2024,
                             prior=lam)
    draws = []
    xo = np.zeros((n, d))
    for it in range(1500):
        G.run(1)
        xg = G.x.cpu().numpy()
        if it < 60:
            ro = oracle.hmc_step(xo, y, 1.0, 0.4, 4, 2024, it, mask=mask, prior_precision=lam)
            xo = ro.x
            assert np.abs(xg - xo).max() <= 1e-12, it
        if it >= 100:
            draws.append(xg.ravel().copy())
    s = np.array(draws)
    acc = G.accepted.item() / 1500
    _log(f"gaussian chain: acceptance {acc:.3f} mean {s.mean():.4f} var {s.var():.4f}")
    assert 0.5 < acc < 1.0
    assert abs(s.mean()) < 0.03
    assert abs(s.var() - 1.0 / lam) < 0.03
    assert abs(np.mean(s ** 4) - 3.0 / lam ** 2) < 0.1


def test_paper_scale_transition():
    """One transition of the paper-scale workload (20 steps) in the spatial
    labelling against the oracle's transition on the same labelling."""
    pr = synth.preset("paper_fp64")
    P = api.MDSProblem(pr.y, pr.d, pr.mask, torch.float64, DEV, order=pr.x)
    x, y, mask = _labelled(P, pr)
    got = _gpu_chain(P, x, pr.sigma, 1e-3, 20, 31, [0])[0]
    ref = oracle.hmc_step(x, y, pr.sigma, 1e-3, 20, 31, 0, mask=mask)
    h0, h1, lu, acc = got["stats"]
    _log(f"paper-scale transition: accepted {ref.accepted}/{bool(acc)} dH {h1 - h0:.3e}")
    assert abs(h0 - ref.energy_start) <= 1e-11 * abs(ref.energy_start)
    assert abs(h1 - ref.energy_end) <= 1e-11 * abs(ref.energy_end)
    assert bool(acc) == ref.accepted
    assert np.abs(got["x"] - ref.x).max() <= 1e-12 * np.abs(ref.x).max()
