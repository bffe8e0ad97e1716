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


def test_tune_batch_records_fastest_row_tile_per_layout(tmp_path, monkeypatch):
    # the batched form's tuner times the persistent launch itself
    monkeypatch.setenv("MDS_TUNE_CACHE", str(tmp_path / "tune.json"))
    e = autotune.tune_batch(torch.float32, 2, 700, reps=3, copies=2)
    cands = autotune.batch_candidates(700, 2, torch.float32)
    assert set(e["by_waves"]) == {str(w) for w in cands}
    for w, r in e["by_waves"].items():
        assert r["ms"] == min(r["candidates_ms"].values())
        assert r["tile_rows"] in cands[int(w)]
    tw, rows = autotune.batch_plan([(700, 2), (650, 2)], torch.float32)
    assert str(tw) in e["by_waves"] and rows == [e["by_waves"][str(tw)]["tile_rows"]] * 2


def test_autotuned_batch_equals_single_calls_and_oracle(tmp_path, monkeypatch):
    # a tuned batch (a common wave layout with row waves, per-problem row
    # tiles from the cache) gives each problem's single-problem result bit
    # for bit, and the oracle's
    monkeypatch.setenv("MDS_TUNE_CACHE", str(tmp_path / "tune.json"))
    monkeypatch.setattr(autotune, "_arch", lambda device=None: "gfx950")
    lay = api.tile_waves(2, 2)
    specs = [dict(n=600, d=2, sigma=0.6, missing=0.1, seed=31),
             dict(n=1400, d=4, sigma=0.4, missing=0.1, seed=32),
             dict(n=900, d=6, sigma=0.9, missing=0.1, seed=33)]
    table = {}
    for s, rows in zip(specs, (32, 128, 64)):
        key = autotune._batch_key("gfx950", torch.float64, s["d"], s["n"])
        table[key] = dict(n=s["n"], pairs=4 * s["n"] * (s["n"] - 1) // 2,
                          by_waves={str(lay): dict(tile_rows=rows, ms=1.0)})
    autotune.save(table)
    probs = [synth.make_problem(**s) for s in specs]
    B = api.MDSBatch([dict(y=p.y, d=p.d, mask=p.mask) for p in probs], torch.float64, "cuda",
                     autotuned=True)
    assert B.tile_waves == lay
    assert [t for t in B.tiles] == [(32, lay), (128, lay), (64, lay)]
    for k, p in enumerate(probs):
        B.set_x(k, p.x)
        B.sigma[k] = p.sigma
    B.eval()
    torch.cuda.synchronize()
    for k, p in enumerate(probs):
        P = api.MDSProblem(p.y, p.d, p.mask, torch.float64, "cuda", *B.tiles[k])
        g, L, ds = P.gradient(B.x[k], p.sigma)
        torch.cuda.synchronize()
        assert torch.equal(g, B.grad[k]) and L.item() == B.loglik[k].item(), k
    ref = oracle.evaluate(probs[1].x, probs[1].y, probs[1].sigma, probs[1].mask)
    got = B.grad[1].cpu().numpy()
    assert abs(B.loglik[1].item() - ref.loglik) <= 1e-12 * abs(ref.loglik)
    assert np.all(np.max(np.abs(got - ref.grad), axis=1) <= 1e-12 * ref.condrow)


def test_batch_autotune_times_the_batch_and_keeps_results(tmp_path, monkeypatch):
    # MDSBatch.autotune() times candidate tilings on the batch itself, keeps
    # the fastest (the library default is a candidate), and the retiled
    # batch still gives each problem's single-problem result bit for bit
    monkeypatch.setenv("MDS_TUNE_CACHE", str(tmp_path / "tune.json"))
    specs = [dict(n=700, d=2, sigma=0.6, missing=0.1, seed=41),
             dict(n=1100, d=4, sigma=0.4, missing=0.1, seed=42),
             dict(n=500, d=6, sigma=0.9, missing=0.1, seed=43)]
    probs = [synth.make_problem(**s) for s in specs]
    B = api.MDSBatch([dict(y=p.y.astype(np.float32), d=p.d, mask=p.mask) for p in probs],
                     torch.float32, "cuda", autotuned=True)
    for k, p in enumerate(probs):
        B.set_x(k, p.x)
        B.sigma[k] = p.sigma
    rec = B.autotune(reps=3)
    assert "library default" in rec["ms"]
    assert rec["ms"][rec["choice"]] == min(rec["ms"].values())
    assert B.tile_waves == rec["tile_waves"]
    B.eval()
    torch.cuda.synchronize()
    for k, p in enumerate(probs):
        P = api.MDSProblem(p.y.astype(np.float32), p.d, p.mask, torch.float32, "cuda",
                           *B.tiles[k])
        g, L, _ = P.gradient(B.x[k], p.sigma)
        torch.cuda.synchronize()
        assert torch.equal(g, B.grad[k]) and L.item() == B.loglik[k].item(), k
    # and the oracle's result (FP32 arithmetic: the FP32 form's tolerance)
    ref = oracle.evaluate(probs[0].x, probs[0].y.astype(np.float32).astype(np.float64),
                          probs[0].sigma, probs[0].mask)
    assert abs(B.loglik[0].item() - ref.loglik) <= 1e-5 * abs(ref.loglik)
