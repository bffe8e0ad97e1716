"""Host-only checks of the C-ABI: the library loads, exports every declared
entry point, and rejects bad arguments before it makes any HIP call (so all
of this runs without a GPU)."""
import ctypes
import os
import re

import pytest
import torch  # noqa: F401  (load torch's HIP runtime first, as the binding does)

from paper_1905_04582_amd import api

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "massivemds.h")

ERR_ARG, ERR_UNSUP, ERR_WS = -1, -2, -3


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(mds_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    names = _declared()
    assert len(names) >= 8
    L = api.lib()
    for nm in names:
        assert hasattr(L, nm), nm


def test_version_and_status_strings():
    L = api.lib()
    assert L.mds_version() >= 10000
    for code, name in [(0, b"MDS_OK"), (-1, b"MDS_ERR_INVALID_ARGUMENT"),
                       (-2, b"MDS_ERR_UNSUPPORTED"), (-3, b"MDS_ERR_WORKSPACE_TOO_SMALL"),
                       (-4, b"MDS_ERR_HIP")]:
        assert L.mds_status_string(code) == name


def test_workspace_query():
    a = api.mds_workspace_bytes(5392, 2, api.MDS_F64)
    b = api.mds_workspace_bytes(5392, 6, api.MDS_F64)
    assert 0 < a < b
    assert api.mds_workspace_bytes(0, 2, api.MDS_F64) == 0
    # explicit tilings: one of tile_rows and 64*tile_waves must divide the other
    for br in (8, 16, 32, 64, 128, 256):
        for w in (1, 2, 4, 8):
            if (64 * w) % br == 0 or br % (64 * w) == 0:
                try:
                    assert api.mds_workspace_bytes(1000, 2, api.MDS_F32, br, w) > 0
                except api.MDSError as e:   # LDS limit for the largest tiles
                    assert e.status == ERR_UNSUP


@pytest.mark.parametrize("args,code", [
    ((10, 0, 0, 0, 0), ERR_UNSUP),        # d = 0
    ((10, 9, 0, 0, 0), ERR_UNSUP),        # d > MDS_MAX_DIM
    ((10, 2, 7, 0, 0), ERR_UNSUP),        # bad dtype
    ((-1, 2, 0, 0, 0), ERR_ARG),          # n < 0
    ((10, 2, 0, 48, 0), ERR_UNSUP),       # tile_rows not in the set
    ((10, 2, 0, 4, 0), ERR_UNSUP),        # tile_rows below the smallest
    ((10, 2, 0, 64, 3), ERR_UNSUP),       # tile_waves not in the set
])
def test_workspace_query_rejects(args, code):
    out = ctypes.c_size_t(0)
    assert api.lib().mds_workspace_bytes(*args, ctypes.byref(out)) == code
    assert api.lib().mds_last_error()  # a detail string was set


FAKE = 1 << 20  # a non-null, well-aligned address that is never dereferenced


def _p(v=FAKE):
    return ctypes.c_void_p(v)


def _loglik(**kw):
    a = dict(n=100, d=2, x=_p(), ldx=2, y=_p(), dt=0, ldy=128, sigma=_p(), out=_p(), ws=_p(),
             wsb=1 << 30, br=0, w=0)
    a.update(kw)
    return api.lib().mds_loglik(a["n"], a["d"], a["x"], a["ldx"], a["y"], a["dt"], a["ldy"],
                                a["sigma"], a["out"], a["ws"], a["wsb"], a["br"], a["w"], None)


@pytest.mark.parametrize("kw,code", [
    (dict(n=-5), ERR_ARG), (dict(d=0), ERR_UNSUP), (dict(d=9), ERR_UNSUP),
    (dict(dt=2), ERR_UNSUP), (dict(x=None), ERR_ARG), (dict(ldx=1), ERR_ARG),
    (dict(y=None), ERR_ARG), (dict(ldy=99), ERR_ARG), (dict(sigma=None), ERR_ARG),
    (dict(out=None), ERR_ARG), (dict(x=_p(FAKE + 4)), ERR_ARG), (dict(y=_p(FAKE + 2)), ERR_ARG),
    (dict(wsb=0), ERR_WS), (dict(ws=None), ERR_ARG), (dict(ws=_p(FAKE + 64)), ERR_ARG),
    (dict(br=100), ERR_UNSUP), (dict(br=64, w=5), ERR_UNSUP),
])
def test_loglik_rejects_before_any_hip_call(kw, code):
    assert _loglik(**kw) == code


def test_gradient_rejects():
    L = api.lib()
    args = [100, 2, _p(), 2, _p(), 0, 128, _p(), None, _p(), 2, None, None, None, _p(),
            1 << 30, 0, 0, None]
    ok = list(args)
    bad = list(ok); bad[9] = None          # grad NULL
    assert L.mds_gradient(*bad) == ERR_ARG
    bad = list(ok); bad[10] = 1            # ldg < d
    assert L.mds_gradient(*bad) == ERR_ARG
    bad = list(ok); bad[8] = _p(FAKE + 1)  # misaligned scale
    assert L.mds_gradient(*bad) == ERR_ARG
    bad = list(ok); bad[13] = _p(FAKE + 4)  # misaligned dlogsigma
    assert L.mds_gradient(*bad) == ERR_ARG
    bad = list(ok); bad[15] = 16           # workspace too small
    assert L.mds_gradient(*bad) == ERR_WS


def test_leapfrog_rejects():
    L = api.lib()
    ok = [100, 2, _p(FAKE), 2, _p(FAKE + 4096), 2, _p(), 0, 128, _p(), None, _p(), None, 20,
          _p(FAKE + 8192), _p(), 0, None, None, _p(), 1 << 30, 0, 0, None]
    bad = list(ok); bad[13] = -1           # n_steps < 0
    assert L.mds_leapfrog(*bad) == ERR_ARG
    bad = list(ok); bad[4] = bad[2]        # p aliases x
    assert L.mds_leapfrog(*bad) == ERR_ARG
    bad = list(ok); bad[11] = None         # step NULL
    assert L.mds_leapfrog(*bad) == ERR_ARG
    bad = list(ok); bad[15] = None         # loglik_io NULL
    assert L.mds_leapfrog(*bad) == ERR_ARG
    bad = list(ok); bad[5] = 1             # ldp < d
    assert L.mds_leapfrog(*bad) == ERR_ARG


def test_prepare_and_log_phi_reject():
    L = api.lib()
    assert L.mds_prepare_y(_p(), 0, 10, None, 0, _p(), 3, 10, 10, None, None, None) == ERR_UNSUP
    assert L.mds_prepare_y(_p(), 0, 9, None, 0, _p(), 0, 10, 10, None, None, None) == ERR_ARG
    assert L.mds_prepare_y(_p(), 0, 10, _p(), 5, _p(), 0, 10, 10, None, None, None) == ERR_ARG
    # in place with a dtype change, and in place with a relabelling
    assert L.mds_prepare_y(_p(), 0, 10, None, 0, _p(), 1, 10, 10, None, None, None) == ERR_ARG
    assert L.mds_prepare_y(_p(), 0, 10, None, 0, _p(), 0, 10, 10, _p(), None, None) == ERR_ARG
    # misaligned permutation
    assert L.mds_prepare_y(_p(), 0, 10, None, 0, _p(FAKE + 4096), 0, 10, 10,
                           _p(FAKE + 3), None, None) == ERR_ARG
    assert L.mds_log_phi(None, None, None, 5, 0, None) == ERR_ARG
    assert L.mds_log_phi(_p(), None, None, -1, 0, None) == ERR_ARG
    assert L.mds_log_phi(_p(), None, None, 5, 4, None) == ERR_UNSUP


def test_check_symmetric_rejects():
    L = api.lib()
    assert L.mds_check_symmetric(_p(), 2, 10, 10, _p(), None) == ERR_UNSUP
    assert L.mds_check_symmetric(_p(), 0, 9, 10, _p(), None) == ERR_ARG
    assert L.mds_check_symmetric(None, 0, 10, 10, _p(), None) == ERR_ARG
    assert L.mds_check_symmetric(_p(), 0, 10, 10, None, None) == ERR_ARG
    assert L.mds_check_symmetric(_p(FAKE + 4), 0, 10, 10, _p(), None) == ERR_ARG
    assert L.mds_status_string(-5) == b"MDS_ERR_NOT_SYMMETRIC"
    # the checked mode validates the same way before any HIP call
    assert L.mds_require_symmetric(_p(), 2, 10, 10, _p(), None) == ERR_UNSUP
    assert L.mds_require_symmetric(_p(), 0, 9, 10, _p(), None) == ERR_ARG
    assert L.mds_require_symmetric(None, 0, 10, 10, _p(), None) == ERR_ARG
    assert L.mds_require_symmetric(_p(), 0, 10, 10, None, None) == ERR_ARG


def test_hmc_rejects():
    L = api.lib()
    nb = ctypes.c_size_t()
    assert L.mds_hmc_workspace_bytes(1000, 2, 0, 0, 0, None) == ERR_ARG
    assert L.mds_hmc_workspace_bytes(1000, 9, 0, 0, 0, ctypes.byref(nb)) == ERR_UNSUP
    assert L.mds_hmc_workspace_bytes(1000, 2, 0, 0, 0, ctypes.byref(nb)) == 0
    g = ctypes.c_size_t()
    assert L.mds_workspace_bytes(1000, 2, 0, 0, 0, ctypes.byref(g)) == 0
    assert nb.value >= g.value + 2 * 1000 * 2 * 8
    assert L.mds_hmc_momentum(10, 2, None, 1, None, _p(), 2, None) == ERR_ARG
    assert L.mds_hmc_momentum(10, 2, None, 1, _p(), None, 2, None) == ERR_ARG
    assert L.mds_hmc_momentum(10, 2, None, 1, _p(), _p(), 1, None) == ERR_ARG
    assert L.mds_hmc_momentum(10, 0, None, 1, _p(), _p(), 2, None) == ERR_UNSUP
    assert L.mds_hmc_momentum(10, 2, None, 1, _p(FAKE + 4), _p(), 2, None) == ERR_ARG
    ws = _p(FAKE + 65536)
    ok = [100, 2, _p(), 2, _p(FAKE + 4096), 0, 128, _p(), None, _p(), None, 20, 7,
          _p(FAKE + 8192), _p(FAKE + 12288), 2, _p(FAKE + 16384), _p(), 0, None, None, ws,
          1 << 30, 0, 0, None]
    bad = list(ok)
    bad[13] = None                                   # no transition counter
    assert L.mds_hmc_step(*bad) == ERR_ARG
    bad = list(ok)
    bad[22] = 16                                     # workspace too small
    assert L.mds_hmc_step(*bad) == ERR_WS
    bad = list(ok)
    bad[21] = _p(FAKE + 65536 + 8)                   # misaligned workspace
    assert L.mds_hmc_step(*bad) == ERR_ARG
    bad = list(ok)
    bad[19] = _p(FAKE + 3)                           # misaligned stats
    assert L.mds_hmc_step(*bad) == ERR_ARG


def test_heldout_and_lpd_reject():
    L = api.lib()
    nb = ctypes.c_size_t()
    assert L.mds_heldout_workspace_bytes(100, None) == ERR_ARG
    assert L.mds_heldout_workspace_bytes(-1, ctypes.byref(nb)) == ERR_ARG
    assert L.mds_heldout_workspace_bytes(100, ctypes.byref(nb)) == 0
    assert nb.value >= 101 * 8 and nb.value % 256 == 0
    ws = _p(FAKE + 65536)
    ok = [_p(), 0, 100, None, 0, _p(FAKE + 4096), 100, 100, _p(FAKE + 8192), ws, nb.value, None]
    assert L.mds_heldout_count(*ok[:8], ok[8], ok[9], 8, None) == ERR_WS
    bad = list(ok)
    bad[1] = 2                                       # unsupported dtype
    assert L.mds_heldout_count(*bad) == ERR_UNSUP
    bad = list(ok)
    bad[6] = 99                                      # ld_heldout < n
    assert L.mds_heldout_count(*bad) == ERR_ARG
    bad = list(ok)
    bad[3], bad[4] = _p(FAKE + 12288), 50            # ld_mask < n
    assert L.mds_heldout_count(*bad) == ERR_ARG
    bad = list(ok)
    bad[8] = None                                    # no count output
    assert L.mds_heldout_count(*bad) == ERR_ARG
    bad = list(ok)
    bad[9] = _p(FAKE + 65536 + 8)                    # misaligned workspace
    assert L.mds_heldout_count(*bad) == ERR_ARG
    fill = ok[:8] + [ws, nb.value, 10, _p(), _p(), _p(), None]
    bad = list(fill)
    bad[10] = -1                                     # negative capacity
    assert L.mds_heldout_fill(*bad) == ERR_ARG
    bad = list(fill)
    bad[11] = None                                   # no row array
    assert L.mds_heldout_fill(*bad) == ERR_ARG
    bad = list(fill)
    bad[13] = _p(FAKE + 4)                           # misaligned y list
    assert L.mds_heldout_fill(*bad) == ERR_ARG
    acc = [10, _p(), _p(), _p(), 2, _p(), 2, _p(), _p(), 1, None]
    bad = list(acc)
    bad[0] = -1
    assert L.mds_lpd_accumulate(*bad) == ERR_ARG
    bad = list(acc)
    bad[4] = 9
    assert L.mds_lpd_accumulate(*bad) == ERR_UNSUP
    bad = list(acc)
    bad[6] = 1                                       # ldx < d
    assert L.mds_lpd_accumulate(*bad) == ERR_ARG
    bad = list(acc)
    bad[7] = None                                    # no sigma
    assert L.mds_lpd_accumulate(*bad) == ERR_ARG
    many = [10, _p(), _p(), _p(), 2, _p(), 2, 20, _p(), 3, _p(), 1, None]
    for k, v, err in ((0, -1, ERR_ARG), (4, 9, ERR_UNSUP), (6, 1, ERR_ARG),
                      (7, -2, ERR_ARG), (8, None, ERR_ARG), (9, -1, ERR_ARG),
                      (5, _p(FAKE + 4), ERR_ARG)):
        bad = list(many)
        bad[k] = v                                   # one bad argument at a time
        assert L.mds_lpd_accumulate_draws(*bad) == err, k
    lb = ctypes.c_size_t()
    assert L.mds_lpd_workspace_bytes(10, None) == ERR_ARG
    assert L.mds_lpd_workspace_bytes(10, ctypes.byref(lb)) == 0 and lb.value % 256 == 0
    fin = [10, _p(), 1, ws, lb.value, _p(), None]
    bad = list(fin)
    bad[2] = 0                                       # no draws
    assert L.mds_lpd_finalize(*bad) == ERR_ARG
    bad = list(fin)
    bad[1] = None                                    # no accumulators
    assert L.mds_lpd_finalize(*bad) == ERR_ARG
    bad = list(fin)
    bad[5] = _p(FAKE + 4)                            # misaligned output
    assert L.mds_lpd_finalize(*bad) == ERR_ARG
    bad = list(fin)
    bad[4] = 8                                       # workspace too small
    assert L.mds_lpd_finalize(*bad) == ERR_WS
    bad = list(fin)
    bad[3] = _p(FAKE + 65536 + 8)                    # misaligned workspace
    assert L.mds_lpd_finalize(*bad) == ERR_ARG


def test_model_flags():
    L = api.lib()
    nb = ctypes.c_size_t()
    assert L.mds_workspace_bytes(1000, 2, 0 | api.MDS_UNTRUNCATED, 0, 0, ctypes.byref(nb)) == 0
    assert L.mds_workspace_bytes(1000, 2, 1 | api.MDS_UNTRUNCATED, 0, 0, ctypes.byref(nb)) == 0
    assert L.mds_workspace_bytes(1000, 2, 0x200, 0, 0, ctypes.byref(nb)) == ERR_UNSUP
    assert L.mds_workspace_bytes(1000, 2, 2 | api.MDS_UNTRUNCATED, 0, 0,
                                 ctypes.byref(nb)) == ERR_UNSUP
    # the flag does not change the tiling or the workspace
    assert api.mds_resolve_tiling(5392, 2, api.MDS_F64 | api.MDS_UNTRUNCATED) == \
        api.mds_resolve_tiling(5392, 2, api.MDS_F64)


def test_resolve_tiling():
    L = api.lib()
    f64, f32 = api.MDS_F64, api.MDS_F32
    assert api.mds_resolve_tiling(1000, 2, f64) == (8, 1)
    assert api.mds_resolve_tiling(1000, 2, f32) == (8, 1)
    tw = api.tile_waves
    assert api.mds_resolve_tiling(2500, 2, f64) == (32, tw(1, 2))
    assert api.mds_resolve_tiling(5392, 2, f64) == (64, tw(1, 4))
    assert api.mds_resolve_tiling(5392, 2, f32) == (64, tw(1, 4))
    assert api.mds_resolve_tiling(5392, 6, f32) == (64, tw(1, 2))
    assert api.mds_resolve_tiling(8000, 2, f64) == (64, tw(1, 2))
    assert api.mds_resolve_tiling(20000, 2, f32) == (128, tw(2, 2))
    assert api.mds_resolve_tiling(20000, 6, f32) == (128, 2)
    assert api.mds_resolve_tiling(5392, 2, f64, 128, 2) == (128, 2)
    r, w = ctypes.c_int32(), ctypes.c_int32()
    assert L.mds_resolve_tiling(100, 2, 0, 48, 1, ctypes.byref(r), ctypes.byref(w)) == ERR_UNSUP
    assert L.mds_resolve_tiling(100, 2, 0, 128, 4, ctypes.byref(r), ctypes.byref(w)) == 0
    assert L.mds_resolve_tiling(100, 9, 0, 0, 0, ctypes.byref(r), ctypes.byref(w)) == ERR_UNSUP
    assert L.mds_resolve_tiling(100, 2, 2, 0, 0, ctypes.byref(r), ctypes.byref(w)) == ERR_UNSUP
    assert L.mds_resolve_tiling(-1, 2, 0, 0, 0, ctypes.byref(r), ctypes.byref(w)) == ERR_ARG
    assert L.mds_resolve_tiling(100, 2, 0, 0, 0, None, ctypes.byref(w)) == ERR_ARG
    # waves down the rows: the value round-trips; a plain count means one row wave
    tw = api.tile_waves(1, 4)
    assert tw == 1 | (4 << 8) and api.split_tile_waves(tw) == (1, 4)
    assert api.split_tile_waves(4) == (4, 1)
    assert api.mds_resolve_tiling(5392, 2, f64, 64, tw) == (64, tw)
    assert api.mds_resolve_tiling(5392, 2, f64, 64, api.tile_waves(2, 1)) == (64, 2)
    # the workspace depends on the tile, not on how its waves split it
    assert api.mds_workspace_bytes(5392, 2, f64, 64, tw) == api.mds_workspace_bytes(5392, 2, f64, 64, 1)
    for br, wv in ((64, api.tile_waves(1, 3)),      # 3 row waves
                   (64, api.tile_waves(4, 4)),      # 16 waves per work-group
                   (16, api.tile_waves(1, 4)),      # 4 rows per wave
                   (64, api.tile_waves(0, 2)),      # no column wave
                   (64, 1 << 16)):                  # undefined bits
        assert L.mds_resolve_tiling(5392, 2, 0, br, wv, ctypes.byref(r), ctypes.byref(w)) == \
            ERR_UNSUP, (br, hex(wv))
    # every tiling the tuner proposes resolves to itself
    import torch
    from paper_1905_04582_amd import autotune
    for br, wv in autotune.candidates(5392, 6, torch.float64):
        assert api.mds_resolve_tiling(5392, 6, f64, br, wv) == (br, wv)


def test_order_and_permute_reject():
    L = api.lib()
    nb = ctypes.c_size_t()
    assert L.mds_order_workspace_bytes(-1, ctypes.byref(nb)) == ERR_ARG
    assert L.mds_order_workspace_bytes(1000, None) == ERR_ARG
    assert L.mds_order_workspace_bytes(1000, ctypes.byref(nb)) == 0
    assert nb.value >= 4 * 4 * 1000 and nb.value % 256 == 0
    assert L.mds_order_workspace_bytes(0, ctypes.byref(nb)) == 0
    ws = _p(FAKE + 65536)
    assert L.mds_spatial_order(100, 0, _p(), 2, _p(), ws, 1 << 20, None) == ERR_UNSUP
    assert L.mds_spatial_order(100, 9, _p(), 9, _p(), ws, 1 << 20, None) == ERR_UNSUP
    assert L.mds_spatial_order(100, 2, _p(), 1, _p(), ws, 1 << 20, None) == ERR_ARG
    assert L.mds_spatial_order(100, 2, None, 2, _p(), ws, 1 << 20, None) == ERR_ARG
    assert L.mds_spatial_order(100, 2, _p(), 2, _p(), _p(FAKE + 8), 1 << 20, None) == ERR_ARG
    assert L.mds_spatial_order(100, 2, _p(), 2, _p(), ws, 16, None) == ERR_WS
    assert L.mds_permute_rows(10, 2, _p(), 2, _p(), 2, _p(), 0, None) == ERR_ARG  # src == dst
    assert L.mds_permute_rows(10, 2, _p(), 1, _p(FAKE + 4096), 2, _p(), 0, None) == ERR_ARG
    assert L.mds_permute_rows(10, 2, _p(), 2, _p(FAKE + 4096), 2, None, 0, None) == ERR_ARG
    assert L.mds_permute_rows(10, 9, _p(), 9, _p(FAKE + 4096), 9, _p(), 0, None) == ERR_UNSUP
    assert L.mds_permute_rows(-1, 2, _p(), 2, _p(FAKE + 4096), 2, _p(), 0, None) == ERR_ARG


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    monkeypatch.setattr(api, "_lib", None)
    monkeypatch.setattr(api, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(RuntimeError, match="no CPU fallback"):
        api.lib()


def test_batch_rejects():
    L = api.lib()
    nb = ctypes.c_size_t(0)
    d = (api.ProblemDesc * 2)()
    for q in d:
        q.n, q.d, q.x, q.ldx, q.y, q.ldy, q.sigma = 100, 2, FAKE, 2, FAKE, 128, FAKE
        q.grad, q.ldg = FAKE, 2
    assert L.mds_batch_workspace_bytes(d, 2, 0, 0, ctypes.byref(nb)) == 0 and nb.value > 0
    assert L.mds_batch_workspace_bytes(d, 0, 0, 0, ctypes.byref(nb)) == ERR_ARG
    assert L.mds_batch_workspace_bytes(None, 2, 0, 0, ctypes.byref(nb)) == ERR_ARG
    assert L.mds_batch_workspace_bytes(d, 2, 5, 0, ctypes.byref(nb)) == ERR_UNSUP
    assert L.mds_batch_workspace_bytes(d, 2, 0, 3, ctypes.byref(nb)) == ERR_UNSUP
    d[1].d = 9
    assert L.mds_batch_workspace_bytes(d, 2, 0, 0, ctypes.byref(nb)) == ERR_UNSUP
    assert b"problem 1" in L.mds_last_error()
    d[1].d = 2
    d[1].ldg = 1
    assert L.mds_batch_workspace_bytes(d, 2, 0, 0, ctypes.byref(nb)) == ERR_ARG
    d[1].ldg = 2
    d[0].tile_rows = 48
    assert L.mds_batch_workspace_bytes(d, 2, 0, 0, ctypes.byref(nb)) == ERR_UNSUP
    d[0].tile_rows = 0
    plan = api.BatchPlan()
    # workspace checks happen before the table upload (no HIP call)
    assert L.mds_batch_init(d, 2, 0, 0, None, 1 << 30, ctypes.byref(plan), None) == ERR_ARG
    assert L.mds_batch_init(d, 2, 0, 0, _p(FAKE + 8), 1 << 30, ctypes.byref(plan), None) == ERR_ARG
    assert L.mds_batch_init(d, 2, 0, 0, _p(), 16, ctypes.byref(plan), None) == ERR_WS
    assert L.mds_batch_init(d, 2, 0, 0, _p(), 1 << 30, None, None) == ERR_ARG
    assert L.mds_batch_eval(None, 1, None) == ERR_ARG
    assert L.mds_batch_eval(ctypes.byref(api.BatchPlan()), 1, None) == ERR_ARG
    # leapfrog fields
    d[1].grad = FAKE + 8192
    d[1].p, d[1].ldp = FAKE + 4096, 1                 # ldp < d
    assert L.mds_batch_workspace_bytes(d, 2, 0, 0, ctypes.byref(nb)) == ERR_ARG
    d[1].ldp = 2
    d[1].step = FAKE + 3                              # misaligned step
    assert L.mds_batch_workspace_bytes(d, 2, 0, 0, ctypes.byref(nb)) == ERR_ARG
    d[1].step = FAKE + 8
    d[1].p = d[1].grad                                # momenta alias the gradient
    assert L.mds_batch_workspace_bytes(d, 2, 0, 0, ctypes.byref(nb)) == ERR_ARG
    d[1].p = FAKE + 4096
    assert L.mds_batch_workspace_bytes(d, 2, 0, 0, ctypes.byref(nb)) == 0
    assert L.mds_batch_leapfrog(None, 20, 0, None) == ERR_ARG
    assert L.mds_batch_leapfrog(ctypes.byref(api.BatchPlan()), 20, 0, None) == ERR_ARG
    # an initialised plan without momenta in every problem is rejected
    pl = api.BatchPlan()
    pl.count, pl.workspace, pl.flags = 2, FAKE, 0
    assert L.mds_batch_leapfrog(ctypes.byref(pl), 20, 0, None) == ERR_ARG
    pl.flags = 1
    assert L.mds_batch_leapfrog(ctypes.byref(pl), -1, 0, None) == ERR_ARG


def test_native_c_program_uses_the_abi_alone(tmp_path):
    # a plain C program (no Python, no torch) compiled against include/ and
    # linked to the library runs the host-side entry points and rejects
    import subprocess
    from paper_1905_04582_amd import build
    exe = build.build_native_check(str(tmp_path / "capi_roundtrip"))
    r = subprocess.run([exe, "cpu"], capture_output=True, text=True, timeout=60)
    assert r.returncode == 0, r.stderr
    assert "capi host checks ok" in r.stdout


def test_gradient_noalloc_validates_before_any_hip_call():
    L = api.lib()
    assert L.mds_noalloc_scratch_bytes() == 32 << 20
    a = [100, 2, _p(), 2, _p(), 0, 128, _p(), None, _p(), 2, None, None, None, 0, 0, None]
    bad = list(a)
    bad[2] = None                                     # x NULL
    assert L.mds_gradient_noalloc(*bad) == ERR_ARG
    bad = list(a)
    bad[10] = 1                                       # ldg < d
    assert L.mds_gradient_noalloc(*bad) == ERR_ARG
    bad = list(a)
    bad[14] = 48                                      # tile_rows not in the set
    assert L.mds_gradient_noalloc(*bad) == ERR_UNSUP
    # a problem whose partial sums exceed the static scratch is refused
    big = [20000, 2, _p(), 2, _p(), 0, 20032, _p(), None, _p(), 2, None, None, None, 0, 0, None]
    assert L.mds_gradient_noalloc(*big) == ERR_WS
    assert b"static scratch" in L.mds_last_error()
