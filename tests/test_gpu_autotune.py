"""Autotuner on the GPU: picks the fastest measured tiling, the cache entry is
used by MDSProblem/MDSBatch, and tuned tilings give the oracle's results."""
import numpy as np
import pytest
import torch

import oracle
from paper_1905_04582_amd import api, autotune, synth

pytestmark = pytest.mark.gpu


def test_tune_records_fastest_and_is_used(tmp_path, monkeypatch):
    monkeypatch.setenv("MDS_TUNE_CACHE", str(tmp_path / "tune.json"))
    e = autotune.tune(torch.float64, 3, 1500, reps=5)
    assert e["ms"] == min(e["candidates_ms"].values())
    assert len(e["candidates_ms"]) == len(autotune.candidates(1500, 3, torch.float64))
    assert autotune.lookup(torch.float64, 3, 1400) == (e["tile_rows"], e["tile_waves"])
    p = synth.make_problem(1400, 3, 0.7, seed=5, missing=0.1)
    P = api.MDSProblem(p.y, 3, p.mask, torch.float64, "cuda", autotuned=True)
    assert (P.tile_rows, P.tile_waves) == (e["tile_rows"], e["tile_waves"])
    g, L, _ = P.gradient(torch.as_tensor(p.x, device="cuda"), p.sigma)
    torch.cuda.synchronize()
    ref = oracle.evaluate(p.x, p.y, p.sigma, p.mask)
    assert abs(L.item() - ref.loglik) <= 1e-12 * abs(ref.loglik)
    assert np.all(np.max(np.abs(g.cpu().numpy() - ref.grad), axis=1) <= 1e-12 * ref.condrow)
