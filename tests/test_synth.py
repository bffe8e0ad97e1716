"""The seeded input generator: reproducible, symmetric, drawn from Eq. (1)."""
import numpy as np
import pytest
from scipy import stats
from scipy.spatial.distance import cdist
from scipy.special import ndtr
import torch

from paper_1905_04582_amd import synth


def test_reproducible_and_seed_sensitive():
    a = synth.make_problem(300, 2, 0.5, seed=3, missing=0.1)
    b = synth.make_problem(300, 2, 0.5, seed=3, missing=0.1)
    c = synth.make_problem(300, 2, 0.5, seed=4, missing=0.1)
    assert np.array_equal(a.y, b.y) and np.array_equal(a.x, b.x)
    assert np.array_equal(a.mask, b.mask)
    assert not np.array_equal(a.y, c.y)


def test_y_symmetric_positive_zero_diagonal():
    p = synth.make_problem(1500, 3, 0.4, seed=5)   # spans two row blocks
    assert np.array_equal(p.y, p.y.T)
    assert np.all(np.diag(p.y) == 0)
    off = p.y[~np.eye(p.n, dtype=bool)]
    assert np.all(off > 0)


def test_y_follows_truncated_normal_model():
    # PIT of y_ij under N(delta_ij, sigma^2) truncated to y > 0 is U(0, 1)
    p = synth.make_problem(400, 2, 0.8, seed=6)
    il = np.tril_indices(p.n, -1)
    delta = cdist(p.x_true, p.x_true)[il]
    y = p.y[il]
    s = p.sigma
    u = (ndtr((y - delta) / s) - ndtr(-delta / s)) / ndtr(delta / s)
    assert stats.kstest(u, "uniform").pvalue > 1e-3


def test_mask_symmetric_at_rate():
    p = synth.make_problem(800, 2, 0.5, seed=7, missing=0.15)
    assert np.array_equal(p.mask, p.mask.T)
    assert np.all(np.diag(p.mask) == 0)
    il = np.tril_indices(p.n, -1)
    rate = p.mask[il].mean()
    assert abs(rate - 0.15) < 0.005


def test_duplicates_are_near_coincident():
    p = synth.make_problem(500, 6, 0.05, seed=8, dup_frac=0.01)
    d = cdist(p.x, p.x)
    np.fill_diagonal(d, np.inf)
    close = np.sum(d.min(axis=1) < 1e-2)
    assert close >= 5   # 5 duplicates, each near its source


def test_batch_specs():
    specs = synth.batch_specs(64, seed=64)
    assert len(specs) == 64
    assert all(500 <= s["n"] <= 8000 and s["d"] in (2, 4, 6) and 0.2 <= s["sigma"] <= 1.0
               for s in specs)
    assert specs == synth.batch_specs(64, seed=64)


@pytest.mark.parametrize("name", ["small_fp64"])
def test_presets(name):
    p = synth.preset(name)
    assert p.x.shape == (p.n, p.d) and p.y.shape == (p.n, p.n)


def test_device_problem_same_recipe():
    # the device-drawn Y (run here on the CPU device) is symmetric, positive
    # off the diagonal, and follows the host recipe's distribution; the
    # locations are the host recipe's exactly
    xt, x, y = synth.device_problem(1500, 2, 0.5, seed=11, device="cpu", block_rows=600)
    host = synth.make_problem(1500, 2, 0.5, seed=11)
    assert np.array_equal(xt, host.x_true) and np.array_equal(x, host.x)
    yn = y.numpy()
    assert np.array_equal(yn, yn.T) and not np.any(np.diag(yn))
    i, j = np.tril_indices(1500, -1)
    assert (yn[i, j] > 0).all()
    dist = np.sqrt(((xt[i] - xt[j]) ** 2).sum(1))
    r_dev = (yn[i, j] - dist) / 0.5
    r_host = (host.y[i, j] - dist) / 0.5
    assert abs(r_dev.mean() - r_host.mean()) < 0.01 and abs(r_dev.std() - r_host.std()) < 0.01
    # deterministic for a seed and block size
    _, _, y2 = synth.device_problem(1500, 2, 0.5, seed=11, device="cpu", block_rows=600)
    assert torch.equal(y, y2)
    _, _, y32 = synth.device_problem(300, 2, 0.5, seed=1, device="cpu", dtype=torch.float32)
    assert y32.dtype == torch.float32


def test_device_problem_missing_pairs():
    _, _, y = synth.device_problem(800, 2, 0.5, seed=3, device="cpu", missing=0.15)
    yn = y.numpy()
    i, j = np.tril_indices(800, -1)
    miss = np.isnan(yn[i, j])
    assert abs(miss.mean() - 0.15) < 0.01
    assert np.array_equal(np.isnan(yn), np.isnan(yn.T)) and not np.isnan(np.diag(yn)).any()
    assert (yn[i, j][~miss] > 0).all()
