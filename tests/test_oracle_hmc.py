"""Pins of the oracle's HMC transition (Section 2.3) and of its random draws.

The generator is pinned by the published known-answer vectors of
Philox4x32-10; the uniform map by its exact end points; the momentum draw
by its distribution (moments, a Kolmogorov-Smirnov distance, independence of
the two Box-Muller outputs, the mass scaling); the Metropolis test by its
limits (a vanishing step is always accepted, an exploding one rejected with
the state, gradient and likelihood restored) and by sampling a Gaussian
target whose variance is known exactly (all pairs missing, prior precision
lambda: every coordinate is N(0, 1/lambda))."""
import json
import math
import os

import numpy as np
import pytest
from scipy import stats

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.json")


def test_philox_known_answers():
    for v in json.load(open(GOLDEN))["vectors"]:
        ctr = [int(h, 16) for h in v["counter"]]
        key = [int(h, 16) for h in v["key"]]
        out = [int(h, 16) for h in v["output"]]
        assert oracle.philox4x32_10(ctr, key).tolist() == out


def test_uniform_open_end_points_and_resolution():
    lo = oracle.uniform_open(0, 0)
    hi = oracle.uniform_open(0xFFFFFFFF, 0xFFFFFFFF)
    assert lo == 2.0 ** -53 and hi == 1.0 - 2.0 ** -53
    # the six low bits of each word are dropped; one unit of b >> 6 is 2^-52
    assert oracle.uniform_open(5 << 6, 0) == oracle.uniform_open((5 << 6) | 63, 63)
    assert oracle.uniform_open(0, 1 << 6) - lo == 2.0 ** -52
    assert oracle.uniform_open(1 << 6, 0) - lo == 2.0 ** -26


def test_momentum_distribution():
    p = oracle.momentum(100000, 2, seed=12345, iteration=7)
    z = p.ravel()
    n = z.size
    assert abs(z.mean()) < 5.0 / math.sqrt(n)
    assert abs(z.var() - 1.0) < 5.0 * math.sqrt(2.0 / n)
    assert stats.kstest(z, "norm").statistic < 1.63 / math.sqrt(n) * 1.5
    # the two outputs of one Box-Muller pair are independent
    assert abs(np.corrcoef(z[0::2], z[1::2])[0, 1]) < 5.0 / math.sqrt(n / 2)
    # other iterations and seeds give other draws
    assert not np.array_equal(p, oracle.momentum(100000, 2, seed=12345, iteration=8))
    assert not np.array_equal(p, oracle.momentum(100000, 2, seed=12346, iteration=7))
    assert np.array_equal(p, oracle.momentum(100000, 2, seed=12345, iteration=7))


def test_momentum_mass_scaling():
    n = 60000
    im = np.empty((n, 2))
    im[:, 0], im[:, 1] = 4.0, 0.25            # M = 1/4 and 4
    p = oracle.momentum(n, 2, seed=3, iteration=1, inv_mass=im)
    assert abs(p[:, 0].var() - 0.25) < 5 * 0.25 * math.sqrt(2.0 / n)
    assert abs(p[:, 1].var() - 4.0) < 5 * 4.0 * math.sqrt(2.0 / n)
    # same normals as the unit-mass draw, scaled by sqrt(M)
    z = oracle.momentum(n, 2, seed=3, iteration=1)
    assert np.allclose(p * np.sqrt(im), z, rtol=1e-15, atol=0)


def _small_problem(n=40, d=2, seed=0):
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((n, d)) * 2.0
    y = np.abs(rng.standard_normal((n, n))) * 3 + 0.1
    y = np.tril(y, -1)
    return x, y + y.T


def test_tiny_step_is_accepted():
    x, y = _small_problem()
    r = oracle.hmc_step(x, y, 0.7, eps=1e-8, n_steps=3, seed=11, iteration=0)
    assert abs(r.energy_end - r.energy_start) < 1e-9 * abs(r.energy_start)
    assert r.accepted and r.log_u < 0.0
    assert not np.array_equal(r.x, x) and np.abs(r.x - x).max() < 1e-6
    ev = oracle.evaluate(r.x, y, 0.7)
    assert np.array_equal(r.grad, ev.grad) and r.loglik == ev.loglik


def test_exploding_step_is_rejected_and_restored():
    x, y = _small_problem()
    r = oracle.hmc_step(x, y, 0.7, eps=5.0, n_steps=10, seed=11, iteration=0,
                        prior_precision=0.5)
    assert not r.accepted
    assert r.log_u >= r.energy_start - r.energy_end or math.isnan(r.energy_end)
    assert np.array_equal(r.x, x)
    ev = oracle.evaluate(x, y, 0.7)
    assert np.array_equal(r.grad, ev.grad - 0.5 * x) and r.loglik == ev.loglik


@pytest.mark.parametrize("it", range(6))
def test_decision_follows_energies(it):
    x, y = _small_problem(seed=it)
    r = oracle.hmc_step(x, y, 0.6, eps=0.05, n_steps=5, seed=99, iteration=it)
    assert r.log_u == math.log(oracle.accept_uniform(99, it))
    assert r.accepted == (r.log_u < r.energy_start - r.energy_end)
    # the energies are those of the leapfrog trajectory from x with the drawn momentum
    tr = oracle.leapfrog(x, oracle.momentum(*x.shape, 99, it), y, 0.6, 0.05, 5)
    assert r.energy_start == tr.energy_start and r.energy_end == tr.energy_end
    if r.accepted:
        assert np.array_equal(r.x, tr.x)


def test_chain_samples_gaussian_target():
    """All pairs missing and prior precision lambda: the target is
    N(0, I / lambda) exactly, so the chain's moments are known."""
    n, d, lam = 25, 2, 2.0
    y = np.ones((n, n))
    mask = np.ones((n, n), np.uint8)
    x = np.zeros((n, d))
    draws, acc = [], 0
    for it in range(1500):
        r = oracle.hmc_step(x, y, 1.0, eps=0.4, n_steps=4, seed=2024, iteration=it,
                            mask=mask, prior_precision=lam)
        x, acc = r.x, acc + r.accepted
        if it >= 100:
            draws.append(x.ravel().copy())
    s = np.array(draws)
    assert 0.5 < acc / 1500 < 1.0
    assert abs(s.mean()) < 0.03
    assert abs(s.var() - 1.0 / lam) < 0.03
    # a wrong momentum scale or acceptance sign would shift the variance
    assert abs(np.mean(s ** 4) - 3.0 / lam ** 2) < 0.1
