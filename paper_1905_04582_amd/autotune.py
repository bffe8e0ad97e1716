"""Tile-shape autotuner for the pair sweep.

For a (Y dtype, D, N bucket) it times every feasible tiling -- rows per tile
(8/16/32/64/128/256) x 64-column groups per tile (1/2/4/8), one dividing the
other, within the LDS budget -- on a problem of that size and keeps the
fastest in a JSON cache keyed by GPU architecture, dtype, D and bucket.

The tuning problem is generated on the device: locations X ~ N(0, 9 I) in
spatial order (as ``MDSProblem(order=...)`` stores a problem) and a random
symmetric Y, evaluated at sigma = 0.5.  The sweep's cost depends on the data
only through the wavefronts that skip the truncation terms, i.e. on how far
apart the locations are relative to sigma.

    python -m paper_1905_04582_amd.autotune --dtype f64 --d 2 --n 5392
    python -m paper_1905_04582_amd.autotune --grid           # the standard grid

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
    code = api.MDS_F64 if dtype == torch.float64 else api.MDS_F32
    out = []
    for br in ROW_TILES:
        for w in WAVE_TILES:
            if (64 * w) % br and br % (64 * w):
                continue
            try:
                api.mds_workspace_bytes(n, d, code, br, w)
            except api.MDSError:
                continue          # exceeds the LDS budget at this D
            out.append((br, w))
    return out


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
    results, sweeps = {}, {}
    for br, w in candidates(n, d, dtype):
        results[f"{br}x{64 * w}"] = time_tiling(x, yp, 0.5, br, w, reps=reps)
        sweeps[f"{br}x{64 * w}"] = time_sweep_only(x, yp, 0.5, br, w, reps=reps)
        if verbose:
            print(f"  {dtype} D={d} N={n} tile {br}x{64 * w}: "
                  f"{results[f'{br}x{64 * w}'] * 1e3:.1f} us "
                  f"(sweep {sweeps[f'{br}x{64 * w}'] * 1e3:.1f} us)", flush=True)
    best = min(results, key=results.get)
    br, cols = (int(v) for v in best.split("x"))
    entry = dict(tile_rows=br, tile_waves=cols // 64, ms=results[best], n=n,
                 candidates_ms=results, sweep_only_ms=sweeps,
                 tuned_at=time.strftime("%Y-%m-%dT%H:%M:%S"))
    table = load(path)
    table[_key(_arch(device), dtype, d, n)] = entry
    save(table, path)
    return entry


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
                    print(f"{_key(_arch(device), dt, d, n)}: best {e['tile_rows']}x"
                          f"{64 * e['tile_waves']} {e['ms'] * 1e3:.1f} us", flush=True)
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--dtype", choices=("f64", "f32"), default="f64")
    ap.add_argument("--d", type=int, default=2)
    ap.add_argument("--n", type=int, default=5392)
    ap.add_argument("--reps", type=int, default=20)
    ap.add_argument("--grid", action="store_true", help="tune the standard (dtype, D, N) grid")
    ap.add_argument("--cache", default=None)
    args = ap.parse_args()
    if args.cache:
        os.environ["MDS_TUNE_CACHE"] = args.cache
    if args.grid:
        tune_grid()
    else:
        dt = torch.float64 if args.dtype == "f64" else torch.float32
        e = tune(dt, args.d, args.n, reps=args.reps, verbose=True)
        print(json.dumps(e))


if __name__ == "__main__":
    main()
