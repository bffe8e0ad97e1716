"""Tile-shape autotuner for the pair sweep.

Single problems: for a (Y dtype, D, N bucket) it times every feasible tiling
-- rows per tile (8/16/32/64/128/256) x 64-column waves across the tile
(1/2/4/8) x waves down its rows (1/2/4/8; at most 8 waves per work-group and
8 rows per wave), rows and columns one dividing the other, within the LDS
budget -- on a problem of that size and keeps the fastest in a JSON cache
keyed by GPU architecture, dtype, D and bucket.

Batches (many problems in one persistent launch): every problem of a batch
shares the work-group's wave layout (tile_waves) and has its own rows per
tile.  For a (dtype, D, N bucket) the batch tuner times the persistent
evaluation of a batch of copies of a problem of that size for every row tile
under each common wave layout and records, per layout, the fastest row tile
and its time.  A batch built with ``autotuned=True`` takes the layout whose
recorded times, scaled by each problem's pairs, add up to the least, and each
problem's fastest row tile under it (``batch_plan``).  ``MDSBatch.autotune()``
then times that plan, the library default and the other layouts on the batch
itself and keeps the fastest (``tune_batch_plan``).

The tuning problems are generated on the device: locations X ~ N(0, 9 I) in
spatial order (as ``MDSProblem(order=...)`` stores a problem) and a random
symmetric Y, evaluated at sigma = 0.5.  The sweep's cost depends on the data
only through the wavefronts that skip the truncation terms, i.e. on how far
apart the locations are relative to sigma.

    python -m paper_1905_04582_amd.autotune --dtype f64 --d 2 --n 5392
    python -m paper_1905_04582_amd.autotune --grid           # the standard grid
    python -m paper_1905_04582_amd.autotune --batch-grid     # the batched form's grid

Lookups (``lookup``) return (tile_rows, tile_waves), or (0, 0) -- the
library's built-in default -- when the cache has no entry.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import time

import torch

from . import api

DEFAULT_CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning.json")
ROW_TILES = (8, 16, 32, 64, 128, 256)
WAVE_TILES = (1, 2, 4, 8)


def cache_path() -> str:
    return os.environ.get("MDS_TUNE_CACHE", DEFAULT_CACHE)


def bucket(n: int) -> int:
    """N bucket: the smallest 2^k or 3 * 2^(k-1) at or above n (minimum 512),
    i.e. half-octave buckets: ..., 4096, 6144, 8192, 12288, ..."""
    b = 512
    while b < n:
        b = b * 3 // 2 if (b & (b - 1)) == 0 else b * 4 // 3
    return b


def _arch(device=None) -> str:
    try:
        return torch.cuda.get_device_properties(device or 0).gcnArchName.split(":")[0]
    except Exception:  # no device
        return "unknown"


def _key(arch, dtype, d, n):
    dt = "f64" if dtype in (torch.float64, "f64") else "f32"
    return f"{arch}|{dt}|D{d}|N{bucket(n)}"


def load(path: str | None = None) -> dict:
    p = path or cache_path()
    if not os.path.exists(p):
        return {}
    with open(p) as f:
        return json.load(f)


def save(table: dict, path: str | None = None):
    p = path or cache_path()
    tmp = p + ".tmp%d" % os.getpid()
    with open(tmp, "w") as f:
        json.dump(table, f, indent=1, sort_keys=True)
    os.replace(tmp, p)


def lookup(dtype, d: int, n: int, device=None, path: str | None = None):
    e = load(path).get(_key(_arch(device), dtype, d, n))
    return (e["tile_rows"], e["tile_waves"]) if e else (0, 0)


def candidates(n: int, d: int, dtype):
    """(tile_rows, tile_waves) of every tiling the library accepts at (n, d)."""
    code = api.MDS_F64 if dtype == torch.float64 else api.MDS_F32
    out = []
    for br in ROW_TILES:
        for w in WAVE_TILES:
            if (64 * w) % br and br % (64 * w):
                continue
            for wr in WAVE_TILES:
                if w * wr > 8 or br // wr < 8:
                    continue
                tw = api.tile_waves(w, wr)
                try:
                    api.mds_resolve_tiling(n, d, code, br, tw)
                except api.MDSError:
                    continue          # exceeds the LDS budget at this D
                out.append((br, tw))
    return out


def label(br: int, tw: int) -> str:
    """'rows x columns / row waves' of a tiling, e.g. '64x64/4'."""
    wc, wr = api.split_tile_waves(tw)
    return f"{br}x{64 * wc}/{wr}"


def _random_problem(n, d, dtype, device, seed=0, ordered=True):
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    x = torch.randn((n, d), generator=g, dtype=torch.float64, device=device) * 3.0
    if ordered:
        x = api.mds_permute_rows(x, api.mds_spatial_order(x))
    y = (torch.randn((n, n), generator=g, dtype=torch.float64, device=device).abs() * 3.0)
    y = torch.tril(y, -1)
    y = (y + y.T).contiguous()
    yp, _ = api.mds_prepare_y(y, dtype, None, count=False)
    del y
    return x, yp


class _RawEvents:
    """hipEvent_t handles for bracketing the sweep kernel alone."""

    def __init__(self):
        import ctypes
        self.ct = ctypes
        self.hip = ctypes.CDLL("libamdhip64.so.7")
        self.hip.hipEventCreate.argtypes = [ctypes.POINTER(ctypes.c_void_p)]
        self.hip.hipEventElapsedTime.argtypes = [ctypes.POINTER(ctypes.c_float),
                                                 ctypes.c_void_p, ctypes.c_void_p]
        self.hip.hipEventDestroy.argtypes = [ctypes.c_void_p]

    def create(self):
        e = self.ct.c_void_p()
        self.hip.hipEventCreate(self.ct.byref(e))
        return e.value

    def elapsed(self, a, b):
        out = self.ct.c_float()
        self.hip.hipEventElapsedTime(self.ct.byref(out), self.ct.c_void_p(a), self.ct.c_void_p(b))
        return float(out.value)

    def destroy(self, e):
        self.hip.hipEventDestroy(self.ct.c_void_p(e))


def time_sweep_only(x, yp, sigma, br, w, reps=20, warmup=3):
    """Median duration (ms) of the sweep kernel alone (finalize excluded)."""
    n, d = x.shape
    code = api.MDS_F64 if yp.dtype == torch.float64 else api.MDS_F32
    ws = api.alloc_workspace(api.mds_workspace_bytes(n, d, code, br, w), x.device)
    g = torch.empty_like(x)
    sig = torch.tensor(sigma, dtype=torch.float64, device=x.device)
    for _ in range(warmup):
        api.mds_gradient(x, yp, sig, ws, grad=g, tile_rows=br, tile_waves=w)
    ev = _RawEvents()
    pairs = [(ev.create(), ev.create()) for _ in range(reps)]
    for a, b in pairs:
        api.mds_set_sweep_events(a, b)
        api.mds_gradient(x, yp, sig, ws, grad=g, tile_rows=br, tile_waves=w)
    api.mds_set_sweep_events(None, None)
    torch.cuda.synchronize()
    ts = sorted(ev.elapsed(a, b) for a, b in pairs)
    for a, b in pairs:
        ev.destroy(a)
        ev.destroy(b)
    return ts[len(ts) // 2]


def time_tiling(x, yp, sigma, br, w, reps=20, warmup=3, want_grad=True):
    n, d = x.shape
    code = api.MDS_F64 if yp.dtype == torch.float64 else api.MDS_F32
    ws = api.alloc_workspace(api.mds_workspace_bytes(n, d, code, br, w), x.device)
    g = torch.empty_like(x)
    L = torch.empty((), dtype=torch.float64, device=x.device)
    sig = torch.tensor(sigma, dtype=torch.float64, device=x.device)

    def once():
        if want_grad:
            api.mds_gradient(x, yp, sig, ws, grad=g, loglik=L, want_dsigma=False,
                             tile_rows=br, tile_waves=w)
        else:
            api.mds_loglik(x, yp, sig, ws, L, tile_rows=br, tile_waves=w)

    for _ in range(warmup):
        once()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(reps)]
    for a, b in ev:
        a.record()
        once()
        b.record()
    torch.cuda.synchronize()
    ts = sorted(a.elapsed_time(b) for a, b in ev)
    return ts[len(ts) // 2]


def tune(dtype, d: int, n: int, device="cuda", reps: int = 20, path: str | None = None,
         verbose: bool = False) -> dict:
    """Time every candidate tiling at (dtype, D, N) and record the fastest."""
    device = torch.device(device)
    x, yp = _random_problem(n, d, dtype, device)
    results, sweeps, tiling = {}, {}, {}
    for br, w in candidates(n, d, dtype):
        k = label(br, w)
        tiling[k] = (br, w)
        results[k] = time_tiling(x, yp, 0.5, br, w, reps=reps)
        sweeps[k] = time_sweep_only(x, yp, 0.5, br, w, reps=reps)
        if verbose:
            print(f"  {dtype} D={d} N={n} tile {k}: {results[k] * 1e3:.1f} us "
                  f"(sweep {sweeps[k] * 1e3:.1f} us)", flush=True)
    best = min(results, key=results.get)
    br, w = tiling[best]
    entry = dict(tile_rows=br, tile_waves=w, ms=results[best], n=n,
                 candidates_ms=results, sweep_only_ms=sweeps,
                 tuned_at=time.strftime("%Y-%m-%dT%H:%M:%S"))
    table = load(path)
    table[_key(_arch(device), dtype, d, n)] = entry
    save(table, path)
    return entry


# ------------------------------------------------------------- batches ----

BATCH_WAVES = ((1, 1), (2, 1), (4, 1), (1, 2), (2, 2), (1, 4), (4, 2), (2, 4), (1, 8))
BATCH_ROWS = (16, 32, 64, 128, 256)
BATCH_COPIES = 4


def _batch_key(arch, dtype, d, n):
    return "batch|" + _key(arch, dtype, d, n)


def batch_candidates(n: int, d: int, dtype):
    """{tile_waves: [tile_rows, ...]} the batched form accepts at (n, d)."""
    code = api.MDS_F64 if dtype == torch.float64 else api.MDS_F32
    out = {}
    for wc, wr in BATCH_WAVES:
        tw = api.tile_waves(wc, wr)
        rows = []
        for br in BATCH_ROWS:
            try:
                api.mds_resolve_tiling(n, d, code, br, tw)
            except api.MDSError:
                continue
            rows.append(br)
        if rows:
            out[tw] = rows
    return out


def time_batch(problems, dtype, tile_waves, reps=10, warmup=3):
    """Median time (ms) of one persistent evaluation (sweep and finalize) of
    an MDSBatch of ``problems`` (dicts with y, d, x, sigma, tile_rows)."""
    B = api.MDSBatch([dict(y=p["y"], d=p["d"], tile_rows=p["tile_rows"]) for p in problems],
                     dtype, problems[0]["y"].device, tile_waves=tile_waves)
    for k, p in enumerate(problems):
        B.x[k].copy_(p["x"])
        B.sigma[k] = p["sigma"]
    for _ in range(warmup):
        B.eval()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(reps)]
    for a, b in ev:
        a.record()
        B.eval()
        b.record()
    torch.cuda.synchronize()
    ts = sorted(a.elapsed_time(b) for a, b in ev)
    del B
    return ts[len(ts) // 2]


def tune_batch(dtype, d: int, n: int, device="cuda", reps: int = 10, copies: int = BATCH_COPIES,
               path: str | None = None, verbose: bool = False) -> dict:
    """Time the persistent batched evaluation of `copies` problems of size n
    for every (common tile_waves, tile_rows) and record the fastest row tile
    per wave layout."""
    device = torch.device(device)
    probs = []
    for c in range(copies):
        x, yp = _random_problem(n, d, torch.float64, device, seed=100 + c)
        probs.append(dict(y=yp, d=d, x=x, sigma=0.5))
    by_waves = {}
    for tw, rows in batch_candidates(n, d, dtype).items():
        times = {}
        for br in rows:
            for p in probs:
                p["tile_rows"] = br
            times[br] = time_batch(probs, dtype, tw, reps=reps)
            if verbose:
                print(f"  batch {dtype} D={d} N={n} waves {api.split_tile_waves(tw)} "
                      f"rows {br}: {times[br] * 1e3:.1f} us", flush=True)
        best = min(times, key=times.get)
        by_waves[str(tw)] = dict(tile_rows=best, ms=times[best], candidates_ms=times)
    entry = dict(n=n, copies=copies, pairs=copies * n * (n - 1) // 2, by_waves=by_waves,
                 tuned_at=time.strftime("%Y-%m-%dT%H:%M:%S"))
    table = load(path)
    table[_batch_key(_arch(device), dtype, d, n)] = entry
    save(table, path)
    return entry


def batch_plan(sizes, dtype, device=None, path: str | None = None, tile_waves: int = 0):
    """Tilings of a batch from the batch tuner's entries: sizes is a list of
    (n, d).  Returns (tile_waves, [tile_rows per problem]) -- the common wave
    layout whose recorded times, each scaled by the problem's pairs over the
    tuning batch's, add up to the least, and every problem's fastest row tile
    under it (0 = the library's default when a problem's bucket has no
    entry).  A given tile_waves is kept and only the row tiles are chosen."""
    table = load(path)
    arch = _arch(device)
    entries = [table.get(_batch_key(arch, dtype, d, n)) for n, d in sizes]
    if tile_waves == 0:
        common = None
        for e in entries:
            if e is not None:
                ks = set(e["by_waves"])
                common = ks if common is None else common & ks
        if common:
            def cost(tw):
                tot = 0.0
                for (n, _), e in zip(sizes, entries):
                    if e is not None:
                        tot += e["by_waves"][tw]["ms"] * (n * (n - 1) / 2) / e["pairs"]
                return tot
            tile_waves = int(min(sorted(common), key=cost))
    rows = []
    for e in entries:
        r = e["by_waves"].get(str(tile_waves)) if (e is not None and tile_waves) else None
        rows.append(int(r["tile_rows"]) if r else 0)
    return tile_waves, rows


def tune_batch_plan(B, reps: int = 5, path: str | None = None) -> dict:
    """Tiles for one batch by timing its whole evaluation (``MDSBatch.autotune``).

    The cached per-bucket entries time batches of copies of one problem
    size; a mixed batch shares one register budget (its largest D) and one
    LDS budget (its largest tile) in a single persistent launch, which those
    entries do not see.  So the candidates -- the library's batch default,
    the cache's plan, and every common wave layout with the cache's row
    tiles or uniform 128-row tiles -- are timed on the batch itself (median
    of ``reps`` evaluations after two warm-up ones) and the fastest is kept.
    Returns the choice and every candidate's time."""
    sizes = [(int(B._descs[k].n), int(B._descs[k].d)) for k in range(B.count)]
    cands = [("library default", 0, None)]
    tw0, rows0 = batch_plan(sizes, B.dtype, B.device, path=path)
    if tw0:
        cands.append(("cache plan", tw0, rows0))
    for wc, wr in BATCH_WAVES:
        tw = api.tile_waves(wc, wr)
        _, rows = batch_plan(sizes, B.dtype, B.device, path=path, tile_waves=tw)
        if any(rows):
            cands.append((f"cache rows, {wc}x{wr} waves", tw, rows))
        cands.append((f"128 rows, {wc}x{wr} waves", tw, [128] * B.count))
    seen, times = set(), {}
    for name, tw, rows in cands:
        key = (tw, tuple(rows) if rows is not None else None)
        if key in seen:
            continue
        seen.add(key)
        try:
            B.retile(tw, rows)
        except api.MDSError:
            continue          # a tiling this batch's LDS budget rejects
        for _ in range(2):
            B.eval()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(reps)]
        for a, b in ev:
            a.record()
            B.eval()
            b.record()
        torch.cuda.synchronize()
        ts = sorted(a.elapsed_time(b) for a, b in ev)
        times[name] = (ts[len(ts) // 2], tw, rows)
    best = min(times, key=lambda k: times[k][0])
    _, tw, rows = times[best]
    B.retile(tw, rows)
    return {"choice": best, "tile_waves": tw, "tile_rows": rows,
            "ms": {k: round(v[0], 4) for k, v in times.items()}}


def tune_batch_grid(dtypes=(torch.float32,), dims=(2, 4, 6), ns=(512, 768, 1024, 1536, 2048,
                                                                    3072, 4096, 6144, 8192),
                    device="cuda", reps=8, verbose=True):
    out = {}
    for dt in dtypes:
        for d in dims:
            for n in ns:
                e = tune_batch(dt, d, n, device=device, reps=reps)
                out[_batch_key(_arch(device), dt, d, n)] = e
                if verbose:
                    best = min(e["by_waves"].items(), key=lambda kv: kv[1]["ms"])
                    print(f"batch {_key(_arch(device), dt, d, n)}: best waves "
                          f"{api.split_tile_waves(int(best[0]))} rows {best[1]['tile_rows']} "
                          f"{best[1]['ms'] * 1e3:.1f} us for {e['copies']} problems", flush=True)
    return out


GRID_N = (1000, 2000, 4000, 5392, 8000, 16000, 20000)


def tune_grid(dtypes=(torch.float64, torch.float32), dims=(2, 4, 6), ns=GRID_N,
              device="cuda", reps=10, verbose=True):
    out = {}
    for dt in dtypes:
        for d in dims:
            for n in ns:
                e = tune(dt, d, n, device=device, reps=reps, verbose=False)
                out[_key(_arch(device), dt, d, n)] = e
                if verbose:
                    print(f"{_key(_arch(device), dt, d, n)}: best "
                          f"{label(e['tile_rows'], e['tile_waves'])} {e['ms'] * 1e3:.1f} us",
                          flush=True)
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--dtype", choices=("f64", "f32"), default="f64")
    ap.add_argument("--d", type=int, default=2)
    ap.add_argument("--n", type=int, default=5392)
    ap.add_argument("--reps", type=int, default=20)
    ap.add_argument("--grid", action="store_true", help="tune the standard (dtype, D, N) grid")
    ap.add_argument("--batch-grid", action="store_true",
                    help="tune the batched form's (D, N bucket) grid (FP32)")
    ap.add_argument("--batch", action="store_true", help="tune the batched form at --dtype/--d/--n")
    ap.add_argument("--cache", default=None)
    args = ap.parse_args()
    if args.cache:
        os.environ["MDS_TUNE_CACHE"] = args.cache
    if args.batch_grid:
        tune_batch_grid()
    elif args.batch:
        dt = torch.float64 if args.dtype == "f64" else torch.float32
        print(json.dumps(tune_batch(dt, args.d, args.n, reps=args.reps, verbose=True)))
    elif args.grid:
        tune_grid()
    else:
        dt = torch.float64 if args.dtype == "f64" else torch.float32
        e = tune(dt, args.d, args.n, reps=args.reps, verbose=True)
        print(json.dumps(e))


if __name__ == "__main__":
    main()
