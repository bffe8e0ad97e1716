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
                wc, _ = api.split_tile_waves(w)
                assert (64 * wc) % br == 0 or br % (64 * wc) == 0
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


def test_candidates_include_row_waves():
    c = autotune.candidates(5392, 2, torch.float64)
    layouts = {api.split_tile_waves(w) for _, w in c}
    assert (1, 4) in layouts and (1, 1) in layouts and (2, 2) in layouts
    for br, w in c:
        wc, wr = api.split_tile_waves(w)
        assert wc * wr <= 8 and br // wr >= 8
    assert autotune.label(64, api.tile_waves(1, 4)) == "64x64/4"


def test_batch_plan_picks_layout_and_rows(tmp_path, monkeypatch):
    path = tmp_path / "t.json"
    monkeypatch.setenv("MDS_TUNE_CACHE", str(path))
    monkeypatch.setattr(autotune, "_arch", lambda device=None: "gfx950")
    w4, w14 = api.tile_waves(4, 1), api.tile_waves(1, 4)
    n1, n2 = 1000, 6000
    p1, p2 = 4 * n1 * (n1 - 1) // 2, 4 * n2 * (n2 - 1) // 2
    table = {
        autotune._batch_key("gfx950", torch.float32, 2, n1): dict(
            n=n1, pairs=p1, by_waves={str(w4): dict(tile_rows=64, ms=1.0),
                                      str(w14): dict(tile_rows=32, ms=0.5)}),
        autotune._batch_key("gfx950", torch.float32, 6, n2): dict(
            n=n2, pairs=p2, by_waves={str(w4): dict(tile_rows=128, ms=4.0),
                                      str(w14): dict(tile_rows=64, ms=6.0)}),
    }
    autotune.save(table)
    # times scale by the problem's pairs over the tuning batch's (4 copies):
    # one problem of each, 0.5/4 + 6.0/4 (1x4) against 1.0/4 + 4.0/4 (4x1)
    assert autotune.batch_plan([(n1, 2), (n2, 6)], torch.float32) == (w4, [64, 128])
    # four of the small one and none of the large: 1x4 wins
    assert autotune.batch_plan([(n1, 2)] * 4, torch.float32) == (w14, [32] * 4)
    # a smaller problem of the large one's bucket (N = 5000: 0.174 of the
    # tuning batch's pairs): 0.5/4 + 6.0 x 0.174 against 1.0/4 + 4.0 x 0.174
    assert autotune.batch_plan([(n1, 2), (5000, 6)], torch.float32)[0] == w4
    # but eight small ones tip it: 8 x 0.5/4 + 1.04 against 8 x 1.0/4 + 0.69
    assert autotune.batch_plan([(n1, 2)] * 8 + [(5000, 6)], torch.float32)[0] == w14
    # an untuned bucket keeps the default row tile; a given layout is kept
    assert autotune.batch_plan([(n1, 2), (20000, 2)], torch.float32) == (w14, [32, 0])
    assert autotune.batch_plan([(n1, 2)], torch.float32, tile_waves=w4) == (w4, [64])
    assert autotune.batch_plan([(n1, 4)], torch.float32) == (0, [0])
