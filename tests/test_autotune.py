"""Autotuner host logic (no GPU): buckets, candidate sets, cache round trip."""
import json

import torch

from paper_1905_04582_amd import api, autotune


def test_buckets():
    assert autotune.bucket(1) == 512 and autotune.bucket(512) == 512
    assert autotune.bucket(513) == 768 and autotune.bucket(769) == 1024
    assert autotune.bucket(5392) == 6144 and autotune.bucket(8000) == 8192
    assert autotune.bucket(20000) == 24576 and autotune.bucket(24577) == 32768
    # the standard grid lands in distinct buckets
    assert len({autotune.bucket(n) for n in autotune.GRID_N}) == len(autotune.GRID_N)


def test_candidates_are_valid_tilings():
    for dt in (torch.float64, torch.float32):
        for d in (1, 2, 6, 8):
            cands = autotune.candidates(5392, d, dt)
            assert cands
            for br, w in cands:
                assert (64 * w) % br == 0 or br % (64 * w) == 0
                code = api.MDS_F64 if dt == torch.float64 else api.MDS_F32
                assert api.mds_workspace_bytes(5392, d, code, br, w) > 0
    # larger D leaves fewer tilings inside the LDS budget
    assert len(autotune.candidates(5392, 8, torch.float64)) <= \
        len(autotune.candidates(5392, 1, torch.float64))


def test_cache_round_trip(tmp_path, monkeypatch):
    path = tmp_path / "t.json"
    monkeypatch.setenv("MDS_TUNE_CACHE", str(path))
    monkeypatch.setattr(autotune, "_arch", lambda device=None: "gfx950")
    assert autotune.lookup(torch.float64, 2, 5392) == (0, 0)
    table = {autotune._key("gfx950", torch.float64, 2, 5392): dict(tile_rows=64, tile_waves=2)}
    autotune.save(table)
    assert json.loads(path.read_text())
    assert autotune.lookup(torch.float64, 2, 5000) == (64, 2)      # same bucket
    assert autotune.lookup(torch.float64, 2, 6500) == (0, 0)       # other bucket
    assert autotune.lookup(torch.float32, 2, 5392) == (0, 0)       # other dtype
