#!/usr/bin/env python3
"""Throughput of the fused MDS log-likelihood + gradient evaluation on one MI355X.

    python bench.py [--steps K] [--warmup W] [--no-cpu] [--gpus 1]

One step = one fused evaluation of the log-likelihood (Eq. 2), its gradient
(Eq. 9) and dL/dsigma on the paper-scale synthetic workload (N = 5392
locations, D = 2, sigma = 0.3, 15% of pairs missing, Y dense FP64 N x N,
inputs resident in device memory).  Prints ONE JSON line.

The locations are relabelled once, at set-up, along a Hilbert curve of the
evaluation point (mds_spatial_order; Y is prepared in that labelling), which
lets most wavefronts skip the truncation terms; the outputs are the same up
to rounding, with the gradient rows in the new labelling.  Besides the FP64
figure (the headline `value`) the line carries the FP32 form on the same
data, both forms in the original labelling, one 20-step leapfrog trajectory,
100 HMC transitions, a 10-step MAP loop through the autograd Function, the
held-out predictive density, the model without
truncation, the batched form (64 problems of uneven N and D, one persistent
launch per evaluation, graph-captured 20-step trajectories of the batch),
the sweep kernel's roofline (each launch of a second pass of the same K
steps timed by HIP events attached to the kernel's own start and end; the
events stay out of the wall-clock pass, whose steps they would slow) and the
serial CPU oracle timed on a bounded sample on this host.

Every timed pass follows W warm-up evaluations, continued until at least
MIN_WARMUP_S seconds of warm-up have run (the GPU clock settles only after
some hundreds of milliseconds of sustained work; `warmup_min_s` in the line).
"""
from __future__ import annotations

import argparse
import ctypes
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
FP64_VALU_TOPS = 39.3216       # 256 CU x 64 FP64 lanes/clk x 2.4 GHz (lane-ops, FMA = 1)
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "sweep_traffic.json")
# sources of the sweep kernel: counter figures in profiles/sweep_traffic.json
# are used only while they and the tiling match
KERNEL_SOURCES = ["mds_sweep.inc.h", "mds_math.h", "mds_coeffs.h", "mds_internal.h", "mds_wave.h",
                  "mds_sweep_f64.hip", "mds_sweep_f32.hip"]


def strip_comments(src: str) -> str:
    """C/C++ source without its comments and with runs of whitespace collapsed
    (string and character literals kept), so that an edit of the comments
    alone leaves the hash of the kernel sources unchanged."""
    out, i, n = [], 0, len(src)
    while i < n:
        c = src[i]
        if c in "\"'":
            j = i + 1
            while j < n and src[j] != c:
                j += 2 if src[j] == "\\" else 1
            out.append(src[i:j + 1])
            i = j + 1
        elif src.startswith("//", i):
            j = src.find("\n", i)
            i = n if j < 0 else j
        elif src.startswith("/*", i):
            j = src.find("*/", i + 2)
            out.append(" ")
            i = n if j < 0 else j + 2
        else:
            out.append(c)
            i += 1
    return " ".join("".join(out).split())


def kernel_source_hash(read=None) -> str:
    """Hash of the sweep kernel's sources, comments aside.  `read(name)`
    returns a source's text (default: the file under csrc/)."""
    if read is None:
        def read(f):
            with open(os.path.join(ROOT, "paper_1905_04582_amd", "csrc", f)) as fh:
                return fh.read()
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(strip_comments(read(f)).encode())
    return h.hexdigest()[:16]


class HipEvents:
    """Raw hipEvent_t handles from the HIP runtime torch already loaded."""

    def __init__(self):
        self.hip = ctypes.CDLL("libamdhip64.so.7")
        self.hip.hipEventCreate.argtypes = [ctypes.POINTER(ctypes.c_void_p)]
        self.hip.hipEventElapsedTime.argtypes = [ctypes.POINTER(ctypes.c_float),
                                                 ctypes.c_void_p, ctypes.c_void_p]
        self.hip.hipEventDestroy.argtypes = [ctypes.c_void_p]

    def create(self):
        e = ctypes.c_void_p()
        if self.hip.hipEventCreate(ctypes.byref(e)) != 0:
            raise RuntimeError("hipEventCreate failed")
        return e.value

    def elapsed_ms(self, a, b) -> float:
        out = ctypes.c_float()
        if self.hip.hipEventElapsedTime(ctypes.byref(out), ctypes.c_void_p(a),
                                        ctypes.c_void_p(b)) != 0:
            raise RuntimeError("hipEventElapsedTime failed")
        return float(out.value)

    def destroy(self, e):
        self.hip.hipEventDestroy(ctypes.c_void_p(e))


# Untimed evaluations run before each timed pass for at least this long (on
# top of the W warm-up steps): the GPU's clock takes a few hundred
# milliseconds of sustained work to settle, and a pass timed before that
# measures the ramp (at N=5392, 20 warm-up evaluations are about 1 ms).
MIN_WARMUP_S = 0.3


def settle(fn, min_s=None):
    """Run fn (one untimed unit of GPU work) until min_s seconds have passed."""
    import torch

    min_s = MIN_WARMUP_S if min_s is None else min_s
    t0 = time.perf_counter()
    while True:
        fn()
        torch.cuda.synchronize()
        if time.perf_counter() - t0 >= min_s:
            return


def timed_evals(P, x, sigma, steps, warmup, events, min_warmup_s=None):
    """K fused evaluations timed by the wall clock between two device
    synchronisations, then K more with HIP events attached to each sweep
    launch (the kernel's own start and end; attaching them costs the step a
    few microseconds, so they stay out of the wall-clock pass).  W warm-up
    evaluations come first, continued until min_warmup_s of warm-up has
    passed.  Returns (wall ms per eval, mean sweep ms, median sweep ms,
    outputs)."""
    import torch
    from paper_1905_04582_amd import api

    g = torch.empty_like(x)
    L = torch.empty((), dtype=torch.float64, device=x.device)
    ds = torch.empty((), dtype=torch.float64, device=x.device)
    sig = torch.tensor(sigma, dtype=torch.float64, device=x.device)
    min_warmup_s = MIN_WARMUP_S if min_warmup_s is None else min_warmup_s
    tw = time.perf_counter()
    for _ in range(warmup):
        P.gradient(x, sig, grad=g, loglik=L, dsigma=ds)
    torch.cuda.synchronize()
    while time.perf_counter() - tw < min_warmup_s:
        for _ in range(50):
            P.gradient(x, sig, grad=g, loglik=L, dsigma=ds)
        torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        P.gradient(x, sig, grad=g, loglik=L, dsigma=ds)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) * 1e3 / steps
    pairs = [(events.create(), events.create()) for _ in range(steps)]
    for a, b in pairs:
        api.mds_set_sweep_events(a, b)
        P.gradient(x, sig, grad=g, loglik=L, dsigma=ds)
    api.mds_set_sweep_events(None, None)
    torch.cuda.synchronize()
    sweep = [events.elapsed_ms(a, b) for a, b in pairs]
    for a, b in pairs:
        events.destroy(a)
        events.destroy(b)
    return wall, sum(sweep) / len(sweep), sorted(sweep)[len(sweep) // 2], (g, L, ds)


def cold_sweep_ms(P, x, sigma, reps, events):
    """Sweep time with the 256 MB Infinity Cache flushed before each call."""
    import torch
    from paper_1905_04582_amd import api

    flush = torch.empty(1 << 29, dtype=torch.uint8, device=x.device)   # 512 MB
    sig = torch.tensor(sigma, dtype=torch.float64, device=x.device)
    out = []
    for _ in range(reps):
        flush.fill_(1)
        a, b = events.create(), events.create()
        api.mds_set_sweep_events(a, b)
        P.gradient(x, sig)
        api.mds_set_sweep_events(None, None)
        torch.cuda.synchronize()
        out.append(events.elapsed_ms(a, b))
        events.destroy(a)
        events.destroy(b)
    del flush
    return sorted(out)[len(out) // 2]


def batch_problems(dev):
    """The batched workload: 64 independent problems, N ~ U[500, 8000], D in
    {2, 4, 6}, sigma ~ U(0.2, 1), 10% missing, FP32 Y drawn on the device.
    Returns (specs, Y list, evaluation points, generating configurations)."""
    import torch

    from paper_1905_04582_amd import synth

    specs = synth.batch_specs(64, seed=64)
    ys, xs, xts = [], [], []
    for sp in specs:
        xtk, xk, yk = synth.device_problem(sp["n"], sp["d"], sp["sigma"], seed=sp["seed"],
                                           device=dev, dtype=torch.float32, missing=sp["missing"])
        ys.append(yk)
        xs.append(xk)
        xts.append(xtk)
    return specs, ys, xs, xts


def only_batch(args):
    """The batched form alone (library default tiles), for profiler runs:
    W + K evaluations of the whole batch, one JSON line."""
    import torch

    from paper_1905_04582_amd import api

    dev = torch.device("cuda:0")
    specs, ys, xs, xts = batch_problems(dev)
    B = api.MDSBatch([dict(y=yk, d=sp["d"], order=xtk) for yk, xtk, sp in zip(ys, xts, specs)],
                     torch.float32, dev)
    del ys
    for k, sp in enumerate(specs):
        B.set_x(k, xs[k])
        B.sigma[k] = sp["sigma"]
    for _ in range(args.warmup):
        B.eval()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        B.eval()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / max(1, args.steps)
    pairs = sum(sp["n"] * (sp["n"] - 1) // 2 for sp in specs)
    print(json.dumps({"form": "batch", "steps": args.steps, "ms_per_batch_eval": ms,
                      "pairs": pairs, "tiles": [list(t) for t in B.tiles]}), flush=True)


def progress(msg):
    print(msg, file=sys.stderr, flush=True)


def n_sweep(args, events):
    """Time per fused evaluation against N (the paper's scaling study over
    randomly sampled 2-D Gaussian points): GPU FP64 and FP32 forms in the
    spatial labelling, the serial oracle where it finishes in seconds, and
    sampled gradient rows against the row oracle at every N."""
    import numpy as np
    import torch

    from paper_1905_04582_amd import api, synth

    dev = torch.device("cuda:0")
    d, sigma = 2, 0.5
    rows_out = []
    for n in args.n_list:
        t0 = time.perf_counter()
        x_true, x, y = synth.device_problem(n, d, sigma, seed=n, device=dev)
        torch.cuda.synchronize()
        gen_s = time.perf_counter() - t0
        progress(f"n-sweep N={n}: Y drawn on the device in {gen_s:.1f} s")
        npairs = n * (n - 1) // 2
        steps = max(5, min(args.steps, int(4e10 / (n * n))))
        warm = max(2, min(args.warmup, steps // 5))
        rec = {"n": n, "pairs": npairs, "steps": steps}
        rng = np.random.default_rng(n)
        rows = np.sort(rng.choice(n, size=min(n, 8), replace=False))
        yrows = y[torch.as_tensor(rows, device=dev)].cpu().numpy() if not args.no_cpu else None
        xd = torch.as_tensor(x, device=dev)
        for name, dt, ybytes in (("fp64", torch.float64, 8), ("fp32", torch.float32, 4)):
            P = api.MDSProblem(y, d, None, dt, dev, order=x_true)
            xr = P.relabel(xd)
            wall, sw, swm, (g, L, ds) = timed_evals(P, xr, sigma, steps, warm, events)
            r = {"ms_per_eval": round(wall, 5), "sweep_ms_mean": round(sw, 5),
                 "evals_per_s": round(1e3 / wall, 3),
                 "y_stream_gbs": round(npairs * ybytes / (sw * 1e-3) / 1e9, 2),
                 "gpairs_per_s": round(npairs / (sw * 1e-3) / 1e9, 3),
                 "tiles": list(api.mds_resolve_tiling(n, d, api._dtype_code(dt)))}
            if yrows is not None:
                import oracle
                gref, _, b = oracle.grad_rows_given(x, yrows, sigma, rows)
                gdev = P.unlabel(g).cpu().numpy()[rows]
                r["sampled_rows_max_err_over_B"] = float(np.max(
                    np.max(np.abs(gdev - gref), axis=1) / b))
            r["loglik"] = L.item()
            rec[name] = r
            progress(f"  {name}: {wall:.4f} ms per evaluation (sweep {sw:.4f} ms)")
            del P, xr, g
        if not args.no_cpu and n <= args.cpu_max_n:
            import oracle
            yh = y.cpu().numpy()
            reps = max(1, int(2e7 / npairs))
            t0 = time.perf_counter()
            for _ in range(reps):
                ev = oracle.evaluate(x, yh, sigma)
            cpu_s = (time.perf_counter() - t0) / reps
            rec["oracle"] = {"s_per_eval": round(cpu_s, 5), "cores": 1, "evals": reps}
            rec["fp64"]["loglik_rel_err"] = abs(rec["fp64"]["loglik"] - ev.loglik) / abs(ev.loglik)
            rec["fp32"]["loglik_rel_err"] = abs(rec["fp32"]["loglik"] - ev.loglik) / abs(ev.loglik)
            rec["gpu_fp64_over_oracle"] = round(cpu_s / (rec["fp64"]["ms_per_eval"] * 1e-3), 1)
            progress(f"  oracle: {cpu_s:.4f} s per evaluation")
            del yh
        rec["y_draw_s"] = round(gen_s, 2)
        rows_out.append(rec)
        del y, xd
        torch.cuda.empty_cache()
    print(json.dumps({
        "metric": "fused loglik+grad evaluation time vs N (D=2, sigma=0.5, no missing pairs)",
        "unit": "ms per evaluation", "n_gpus": 1, "data": "synthetic",
        "config": {"workload": "N sweep: X_true ~ N(0, I_2)*3, y_ij truncated N(delta_ij, "
                               "0.25) drawn on the device, evaluation point X_true + "
                               "N(0, 0.01); locations relabelled in Hilbert order",
                   "d": d, "sigma": sigma},
        "points": rows_out}), flush=True)


def tile_trace(out_path, events, tile_rows=0, tile_waves=0):
    """Per-wave timeline of the FP64 sweep at N = 5392 (relabelled; default
    tiles unless given): start and end clock and hardware slot of every wave
    (mds_set_tile_trace), in one evaluation after the warm-up."""
    import numpy as np
    import torch

    from paper_1905_04582_amd import api, synth

    dev = torch.device("cuda:0")
    prob = synth.preset("paper_fp64")
    n = prob.n
    P = api.MDSProblem(prob.y, 2, prob.mask, torch.float64, dev, order=prob.x_true,
                       tile_rows=tile_rows, tile_waves=tile_waves)
    br, tw = api.mds_resolve_tiling(n, 2, api.MDS_F64, tile_rows, tile_waves)
    wc, wr = api.split_tile_waves(tw)
    w = wc * wr
    ntiles = api.tile_count(n, br, wc)
    buf = torch.zeros(ntiles * w * 3, dtype=torch.int64, device=dev)
    xr = P.relabel(torch.as_tensor(prob.x, device=dev))
    sig = torch.tensor(prob.sigma, dtype=torch.float64, device=dev)
    settle(lambda: P.gradient(xr, sig))
    api.mds_set_tile_trace(buf)
    P.gradient(xr, sig)
    torch.cuda.synchronize()
    api.mds_set_tile_trace(None)
    tr = buf.view(ntiles, w, 3).cpu().numpy()
    t0 = tr[:, :, 0].min()
    s, e = (tr[:, :, 0] - t0) * 0.01, (tr[:, :, 1] - t0) * 0.01      # 100 MHz clock -> us
    hw = tr[:, :, 2]
    xcd = (np.arange(ntiles) % 8)[:, None]
    slot = xcd * 4096 + ((hw >> 13) & 7) * 512 + ((hw >> 12) & 1) * 256 + \
        ((hw >> 8) & 15) * 4 + ((hw >> 4) & 3)
    _, per_simd = np.unique(slot, return_counts=True)
    ts = np.linspace(0.0, float(e.max()), 15)
    dur = e - s
    busy = np.sort(np.concatenate([s.ravel(), e.ravel()]))
    out = {"n": n, "tile_rows": br, "column_waves": wc, "row_waves": wr, "tiles": ntiles,
           "waves": int(ntiles * w), "span_us": round(float(e.max()), 2),
           "last_start_us": round(float(s.max()), 2),
           "active_waves_at": {f"{t:.1f}": int(((s <= t) & (e > t)).sum()) for t in ts},
           "waves_per_simd": {"min": int(per_simd.min()), "max": int(per_simd.max()),
                              "mean": round(float(per_simd.mean()), 2)},
           "wave_us": {"mean": round(float(dur.mean()), 2), "p50": round(float(np.median(dur)), 2),
                       "p90": round(float(np.percentile(dur, 90)), 2),
                       "max": round(float(dur.max()), 2)},
           "wave_busy_us_total": round(float(dur.sum()), 1), "events": int(busy.size)}
    if out_path:
        with open(out_path, "w") as f:
            json.dump(out, f, indent=1)
    print(json.dumps(out), flush=True)
    return out



# bytes one lpd accumulation pass moves per held-out pair: row and column
# (int32 each), y (FP64), and the 2-double state read and written
LPD_BYTES_PER_PAIR_PASS = 4 + 4 + 8 + 16 + 16


def heldout_lpd(prob, xd, sigma, dev, draws=100, per_pass=10):
    """The held-out predictive density of 10% of the pairs of `prob` at the
    locations `xd` (original labelling): compaction time, then `draws` draws
    one per pass and `draws` draws `per_pass` per pass.  Returns the bench
    record (with the HBM figures of the single-draw pass), the lpd of the
    single-draw accumulator and the held-out mask."""
    import numpy as np
    import torch
    from paper_1905_04582_amd import api, synth
    n = prob.n
    held = synth.symmetric_mask(n, 0.10, np.random.Generator(np.random.PCG64(prob.seed + 9)))
    y_d = torch.as_tensor(prob.y, device=dev)
    held_d = torch.as_tensor(held, device=dev)
    mask_d = torch.as_tensor(prob.mask, device=dev)
    api.HeldOutPairs(y_d, held_d, mask_d, dev)          # warm: allocator and code paths
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    H = api.HeldOutPairs(y_d, held_d, mask_d, dev)
    torch.cuda.synchronize()
    setup_ms = (time.perf_counter() - t0) * 1e3
    sig_d = torch.tensor(sigma, dtype=torch.float64, device=dev)
    for _ in range(5):
        H.add_draw(xd, sig_d)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(draws):
        H.add_draw(xd, sig_d)
    torch.cuda.synchronize()
    draw_ms = (time.perf_counter() - t0) * 1e3 / draws
    lpd_val = H.lpd().item()
    # the same draws folded per_pass to a pass (the per-pair state read and
    # written once per pass), in a second accumulator
    xs = xd.unsqueeze(0).expand(per_pass, -1, -1).contiguous()
    sigs = sig_d.expand(per_pass).contiguous()
    Hb = api.HeldOutPairs(y_d, held_d, mask_d, dev)
    Hb.add_draws(xs, sigs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(draws // per_pass):
        Hb.add_draws(xs, sigs)
    torch.cuda.synchronize()
    batched_ms = (time.perf_counter() - t0) * 1e3 / draws
    pass_bytes = H.m * LPD_BYTES_PER_PAIR_PASS
    achieved = pass_bytes / (draw_ms * 1e-3) / 1e9
    rec = {"pairs": H.m, "draws": H.draws, "compaction_ms": round(setup_ms, 3),
           "ms_per_draw": round(draw_ms, 5),
           f"ms_per_draw_{per_pass}_per_pass": round(batched_ms, 5),
           "pairs_per_s": round(H.m / (draw_ms * 1e-3), 1), "lpd": lpd_val,
           "roofline": {"bound": "hbm", "kernel": "lpd_accumulate_kernel (one draw per pass)",
                        "algorithmic_bytes_per_launch": pass_bytes,
                        "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": round(achieved / HBM_PEAK_GBS, 4)}}
    return rec, lpd_val, held


def main():
    global MIN_WARMUP_S
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--min-warmup-s", type=float, default=MIN_WARMUP_S,
                    help="least seconds of warm-up before each timed pass (0: W steps only, "
                         "e.g. under a profiler)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-evals", type=int, default=10)
    ap.add_argument("--only", choices=("fp64", "fp32", "fp64-plain", "fp32-plain", "lpd", "batch"),
                    default=None,
                    help="time one form only (for profiler runs); prints a short JSON line")
    ap.add_argument("--n-sweep", action="store_true",
                    help="time the evaluation against N instead (one JSON line with a point "
                         "per N)")
    ap.add_argument("--n-list", type=lambda v: [int(t) for t in v.split(",")],
                    default=[1000, 2000, 5000, 10000, 20000, 50000, 100000])
    ap.add_argument("--cpu-max-n", type=int, default=20000,
                    help="largest N at which the N sweep times the serial oracle")
    ap.add_argument("--tile-trace", default=None, metavar="JSON",
                    help="write the per-wave timeline of one FP64 sweep (diagnostics)")
    ap.add_argument("--tile-rows", type=int, default=0, help="tile rows for --tile-trace")
    ap.add_argument("--tile-waves", type=int, default=0,
                    help="tile_waves (MDS_TILE_WAVES(wc, wr)) for --tile-trace")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MB",
                    help="only run plain device copies of MB megabytes (calibrates the HBM "
                         "byte counters) and exit")
    args = ap.parse_args()
    MIN_WARMUP_S = max(0.0, args.min_warmup_s)
    if args.copy_calibration:
        import torch
        nbytes = args.copy_calibration << 20
        src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_per_launch": nbytes}), flush=True)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the MDS sweep is built and measured on a "
              "single MI355X (see the sharding design); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    if args.tile_trace:
        import torch
        torch.cuda.init()
        tile_trace(args.tile_trace, None, args.tile_rows, args.tile_waves)
        return
    if args.n_sweep:
        import torch
        torch.cuda.init()      # the HIP runtime torch loads is the one the events use
        n_sweep(args, HipEvents())
        return
    if args.only == "batch":
        only_batch(args)
        return

    import numpy as np
    import torch

    from paper_1905_04582_amd import api, synth

    dev = torch.device("cuda:0")
    prob = synth.preset("paper_fp64")
    n, d, sigma = prob.n, prob.d, prob.sigma
    x = torch.as_tensor(prob.x, device=dev).contiguous()
    npairs = n * (n - 1) // 2
    if args.only == "lpd":
        # the held-out density alone (for profiler runs), at the evaluation point
        rec, _, _ = heldout_lpd(prob, x, sigma, dev, draws=max(10, args.steps))
        print(json.dumps({"form": "lpd", **rec}), flush=True)
        return
    events = HipEvents()

    # set-up (not timed as a step): relabel the locations in Hilbert order of
    # the configuration that generated Y and prepare Y in that labelling; the
    # evaluation point (that configuration moved by N(0, 0.1^2) per
    # coordinate) is not the ordering point, as in a chain that was ordered
    # once at its start
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    P64 = api.MDSProblem(prob.y, d, prob.mask, torch.float64, dev, order=prob.x_true)
    torch.cuda.synchronize()
    setup_ms = (time.perf_counter() - t0) * 1e3
    P32 = api.MDSProblem(prob.y, d, prob.mask, torch.float32, dev, order=prob.x_true)
    xr = P64.relabel(x)
    forms = {"fp64": (P64, xr), "fp32": (P32, xr)}
    if args.only is None or args.only.endswith("plain"):
        forms["fp64-plain"] = (api.MDSProblem(prob.y, d, prob.mask, torch.float64, dev), x)
        forms["fp32-plain"] = (api.MDSProblem(prob.y, d, prob.mask, torch.float32, dev), x)
    m_obs = int(P64.m_obs.item())
    # the tiles the default launch uses, per form
    tiles = {f: list(api.mds_resolve_tiling(n, d, c)) for f, c in
             (("fp64", api.MDS_F64), ("fp32", api.MDS_F32))}

    if args.only:
        P, xx = forms[args.only]
        wall, sweep, sweep_med, _ = timed_evals(P, xx, sigma, args.steps, args.warmup, events)
        print(json.dumps({"form": args.only, "steps": args.steps, "ms_per_step": wall,
                          "sweep_ms_mean": sweep, "sweep_ms_median": sweep_med}), flush=True)
        return

    res = {k: timed_evals(P, xx, sigma, args.steps, args.warmup, events)
           for k, (P, xx) in forms.items()}
    wall64, sweep64, sweep64_med, (g64r, L64, ds64) = res["fp64"]
    wall32, sweep32, sweep32_med, (g32r, L32, ds32) = res["fp32"]
    g64 = P64.unlabel(g64r)
    cold64 = cold_sweep_ms(P64, xr, sigma, 10, events)
    cold32 = cold_sweep_ms(P32, xr, sigma, 10, events)

    # one 20-step leapfrog trajectory (step 1e-3, unit mass), FP64
    mom = P64.relabel(np.random.default_rng(7).standard_normal((n, d)))
    xl, pl = xr.clone(), mom.clone()
    gio = torch.empty_like(xl)
    lio = torch.empty((), dtype=torch.float64, device=dev)
    P64.leapfrog(xl, pl, sigma, 1e-3, 20, gio, lio)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    reps = 5
    for _ in range(reps):
        xl.copy_(xr)
        pl.copy_(mom)
        P64.leapfrog(xl, pl, sigma, 1e-3, 20, gio, lio)
    torch.cuda.synchronize()
    traj_ms = (time.perf_counter() - t0) * 1e3 / reps

    # 100 HMC transitions of 20 leapfrog steps (step 1e-3, unit mass), FP64,
    # replayed as a captured graph of 10 transitions; the chain starts at the
    # evaluation point
    from paper_1905_04582_amd import graphs
    chain = graphs.HMCChainGraph(P64, xr, n_steps=20, sigma=sigma, step=1e-3, seed=1905,
                                 transitions_per_graph=10)
    chain.run(1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    chain.run(10)
    torch.cuda.synchronize()
    hmc_ms = (time.perf_counter() - t0) * 1e3 / 100
    hmc_acc = chain.accepted.item() / 110

    # differentiation form: the torch.autograd.Function over (X, ln sigma),
    # a 10-step gradient-ascent MAP loop (forward = loglik-only sweep,
    # backward = one gradient sweep scaled by the upstream gradient)
    from paper_1905_04582_amd import autograd
    ls0 = torch.tensor(float(np.log(sigma)), dtype=torch.float64, device=dev)
    # step sizes for this workload's gradient scale (rows ~ 1e3-1e4, dL/d ln sigma ~ 1e6)
    autograd.map_ascent(P64, xr, ls0, steps=2, lr_x=1e-6, lr_s=1e-9)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, _, map_trace = autograd.map_ascent(P64, xr, ls0, steps=10, lr_x=1e-6, lr_s=1e-9)
    torch.cuda.synchronize()
    map_ms = (time.perf_counter() - t0) * 1e3 / 10
    map_l = map_trace.cpu().numpy()
    autograd_map = {"steps": 10, "ms_per_step": round(map_ms, 4),
                    "loglik_first_last": [float(map_l[0]), float(map_l[-1])],
                    "step": "forward loglik sweep + backward gradient sweep + torch update"}

    # held-out predictive density: 10% of the pairs held out (symmetric
    # Bernoulli), compacted once, then one accumulation pass per posterior
    # draw (the chain's final state stands in for the draws) and one finalize
    xd = P64.unlabel(chain.x)
    heldout, lpd_val, held = heldout_lpd(prob, xd, sigma, dev)

    # batched form: 64 independent problems, N ~ U[500, 8000], D in {2, 4, 6},
    # sigma ~ U(0.2, 1), 10% missing, FP32 Y drawn in device memory; one
    # persistent sweep and one finalize per evaluation of the whole batch, and
    # 20-step leapfrog trajectories of every problem captured as one graph
    specs, ys, xs, xts = batch_problems(dev)
    # the batch with its tiles picked by the batch autotuner: the plan from
    # the cached per-(D, N bucket) entries, then MDSBatch.autotune() timing
    # that plan, the library default and the other wave layouts on this
    # batch; timed beside the library's batch default below
    Bt = api.MDSBatch([dict(y=yk, d=sp["d"], order=xtk) for yk, xtk, sp in zip(ys, xts, specs)],
                      torch.float32, dev, autotuned=True)
    for k, sp in enumerate(specs):
        Bt.set_x(k, xs[k])
        Bt.sigma[k] = sp["sigma"]
    settle(Bt.eval)
    t0 = time.perf_counter()
    tune_rec = Bt.autotune()
    tune_s = time.perf_counter() - t0
    settle(Bt.eval)
    t0 = time.perf_counter()
    for _ in range(20):
        Bt.eval()
    torch.cuda.synchronize()
    tuned_ms = (time.perf_counter() - t0) * 1e3 / 20
    tuned_tw = api.split_tile_waves(Bt.tile_waves) if Bt.tile_waves else None
    tuned_rows = sorted(set(int(t[0]) for t in Bt.tiles))
    del Bt
    torch.cuda.empty_cache()
    B = api.MDSBatch([dict(y=yk, d=sp["d"], order=xtk) for yk, xtk, sp in zip(ys, xts, specs)],
                     torch.float32, dev)
    del ys
    torch.cuda.empty_cache()
    for k, sp in enumerate(specs):
        B.set_x(k, xs[k])
        B.sigma[k] = sp["sigma"]
    bpairs = sum(sp["n"] * (sp["n"] - 1) // 2 for sp in specs)
    settle(B.eval)
    breps = 20
    t0 = time.perf_counter()
    for _ in range(breps):
        B.eval()
    torch.cuda.synchronize()
    batch_ms = (time.perf_counter() - t0) * 1e3 / breps
    ev_pairs = [(events.create(), events.create()) for _ in range(breps)]
    for a, b in ev_pairs:
        api.mds_set_sweep_events(a, b)
        B.eval()
    api.mds_set_sweep_events(None, None)
    torch.cuda.synchronize()
    bsweep = sorted(events.elapsed_ms(a, b) for a, b in ev_pairs)
    bsweep_mean = sum(bsweep) / len(bsweep)
    for a, b in ev_pairs:
        events.destroy(a)
        events.destroy(b)
    gen = torch.Generator(device=dev)
    gen.manual_seed(7)
    for k in range(B.count):
        B.p[k].copy_(torch.randn(B.p[k].shape, generator=gen, dtype=torch.float64, device=dev))
    B.step.fill_(1e-3)
    B.leapfrog(0)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        B.leapfrog(20, cache_valid=True)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    G = torch.cuda.CUDAGraph()
    with torch.cuda.graph(G):
        B.leapfrog(20, cache_valid=True)
    G.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(5):
        G.replay()
    torch.cuda.synchronize()
    btraj_ms = (time.perf_counter() - t0) * 1e3 / 5
    batched = {
        "problems": B.count, "pairs": bpairs, "dtype": "f32",
        "ms_per_batch_eval": round(batch_ms, 4),
        "sweep_ms_mean": round(bsweep_mean, 4),
        "gpairs_per_s": round(bpairs / (batch_ms * 1e-3) / 1e9, 2),
        "y_stream_gbs": round(bpairs * 4 / (bsweep_mean * 1e-3) / 1e9, 1),
        "y_stream_frac": round(bpairs * 4 / (bsweep_mean * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        "leapfrog_20_steps_graph_ms": round(btraj_ms, 3),
        "tiles": "library batch default (128-row tiles, 2 column waves)",
        "autotuned": {"ms_per_batch_eval": round(tuned_ms, 4),
                      "gpairs_per_s": round(bpairs / (tuned_ms * 1e-3) / 1e9, 2),
                      "choice": tune_rec["choice"], "tile_waves": tuned_tw,
                      "tile_rows": tuned_rows, "tuning_s": round(tune_s, 2),
                      "candidates_ms": tune_rec["ms"],
                      "speedup_vs_default": round(batch_ms / tuned_ms, 3)},
        "workload": "64 problems, N ~ U[500, 8000], D in {2,4,6}, sigma ~ U(0.2,1), 10% "
                    "missing, FP32 Y drawn in device memory; each problem relabelled in "
                    "the spatial order of its generating configuration and evaluated at "
                    "that configuration moved by N(0, 0.1^2)",
    }
    del B, G, xs, xts
    torch.cuda.empty_cache()

    # the model without truncation (the paper's comparison of the two): the
    # same sweep with the special functions left out, and the oracle's time
    # for it on one core
    abl = {}
    for name, dt in (("fp64", torch.float64), ("fp32", torch.float32)):
        Pu = api.MDSProblem(prob.y, d, prob.mask, dt, dev, order=prob.x_true, truncated=False)
        w, sw, _, _ = timed_evals(Pu, xr, sigma, args.steps, args.warmup, events)
        abl[name] = {"ms_per_step": round(w, 5), "sweep_ms_mean": round(sw, 5)}
        del Pu

    # algorithmic traffic of one sweep: the strict lower triangle of Y once
    # (X in and the partial sums out are under 0.1% of it)
    y_bytes64 = npairs * 8
    y_bytes32 = npairs * 4
    gbs64 = y_bytes64 / (sweep64 * 1e-3) / 1e9
    gbs32 = y_bytes32 / (sweep32 * 1e-3) / 1e9

    # HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, calibrated against a
    # plain copy) and the VALU-busy fraction, from the committed counter runs
    # of this same kernel source; null once the kernel has changed
    counters = {}
    if os.path.exists(TRAFFIC_FILE):
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
        if (t.get("kernel_source_sha") == kernel_source_hash() and t.get("n") == n
                and t.get("tiles") == tiles):
            counters = t
    c64, c32 = counters.get("fp64", {}), counters.get("fp32", {})
    traffic = c64.get("traffic_bytes_per_launch")

    def busy_warm(c, sweep_ms):
        # VALU-busy fraction of the warm launch: the counter run's VALU
        # quad-cycles over every SIMD's cycles in the bench's own mean launch
        # time at the 2.4 GHz peak clock (a lower bound: a slower clock gives
        # fewer cycles).  The counter runs' own fraction (valu_busy_frac) is
        # taken over their launches' own durations at the same clock; those
        # launches last longer than warm ones.
        a = c.get("sq_active_inst_valu")
        return round(4 * a / (1024 * 2.4e9 * sweep_ms * 1e-3), 4) if a else None

    plain = {}
    for k in ("fp64-plain", "fp32-plain"):
        w, sw, swm, _ = res[k]
        plain[k] = {"ms_per_step": round(w, 5), "sweep_ms_mean": round(sw, 5)}

    out = {
        "metric": "loglik+grad evals/sec at N=5392,D=2 (FP64 vs FP32) + achieved HBM GB/s",
        "value": round(1e3 / wall64, 3),
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "warmup_min_s": MIN_WARMUP_S,
        "ms_per_step": round(wall64, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "paper-scale plain method: N=5392 D=2 sigma=0.3, 15% of pairs "
                               "missing (symmetric Bernoulli), Y dense FP64 5392x5392, one fused "
                               "loglik+gradient+dL/dsigma evaluation per step; locations "
                               "relabelled once at set-up in Hilbert order of the generating "
                               "configuration, evaluated at that configuration moved by "
                               "N(0, 0.1^2) per coordinate",
                   "n": n, "d": d, "sigma": sigma, "pairs": npairs, "observed_pairs": m_obs,
                   "tiles_rows_x_64cols": tiles, "seed": prob.seed,
                   "setup_ms_order_and_prepare": round(setup_ms, 3)},
        "roofline": {
            "bound": "hbm", "kernel": "sweep_kernel<double,2,true>",
            "achieved": round(gbs64, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(gbs64 / HBM_PEAK_GBS, 4), "traffic": traffic,
            "algorithmic_bytes_per_launch": y_bytes64,
            "valu_busy_frac": c64.get("valu_busy_frac"),
            "valu_busy_frac_warm_min": busy_warm(c64, sweep64),
            "counters": "profiles/sweep_traffic.json" if counters else None,
            "sweep_ms_mean": round(sweep64, 5), "sweep_ms_median": round(sweep64_med, 5),
            "sweep_ms_cold_median": round(cold64, 5),
        },
        # the binding resource: issued FP64 VALU lane-operations (an FMA counts
        # once) per second, from the counter run's instruction count of this
        # kernel source, against 256 CUs x 4 SIMDs x 16 FP64 lanes x 2.4 GHz
        "roofline_alu": {
            "bound": "alu", "kernel": "sweep_kernel<double,2,true>",
            "achieved": (round(c64["sq_insts_valu"] * 64 / (sweep64 * 1e-3) / 1e12, 3)
                         if c64.get("sq_insts_valu") else None),
            "peak": FP64_VALU_TOPS, "unit": "T lane-op/s",
            "frac": (round(c64["sq_insts_valu"] * 64 / (sweep64 * 1e-3) / 1e12 / FP64_VALU_TOPS, 4)
                     if c64.get("sq_insts_valu") else None),
            "valu_insts_per_launch": c64.get("sq_insts_valu"),
        },
        "fp32_form": {
            "value": round(1e3 / wall32, 3), "unit": "evals/s", "ms_per_step": round(wall32, 5),
            "speedup_vs_fp64": round(wall64 / wall32, 3), "sweep_ms_mean": round(sweep32, 5),
            "sweep_ms_cold_median": round(cold32, 5),
            "y_stream_gbs": round(gbs32, 2), "y_stream_frac": round(gbs32 / HBM_PEAK_GBS, 4),
            "traffic": c32.get("traffic_bytes_per_launch"),
            "valu_busy_frac": c32.get("valu_busy_frac"),
            "valu_busy_frac_warm_min": busy_warm(c32, sweep32),
            "loglik_rel_diff_vs_fp64": abs(L32.item() - L64.item()) / abs(L64.item()),
            # issued VALU lane-operations (FP32 without packed math issues
            # at the FP64 rate: 16 lanes per SIMD per clock)
            "roofline_alu": {
                "bound": "alu", "kernel": "sweep_kernel<float,2,true>",
                "achieved": (round(c32["sq_insts_valu"] * 64 / (sweep32 * 1e-3) / 1e12, 3)
                             if c32.get("sq_insts_valu") else None),
                "peak": FP64_VALU_TOPS, "unit": "T lane-op/s",
                "frac": (round(c32["sq_insts_valu"] * 64 / (sweep32 * 1e-3) / 1e12 /
                               FP64_VALU_TOPS, 4) if c32.get("sq_insts_valu") else None),
                "valu_insts_per_launch": c32.get("sq_insts_valu"),
            },
        },
        "original_labelling": plain,
        "untruncated_model": abl,
        "autograd_map": autograd_map,
        "heldout_lpd": heldout,
        "batched_form": batched,
        # the trajectory starts without a cached gradient: one evaluation at
        # the start, then one per step
        "leapfrog": {"steps": 20, "step_size": 1e-3, "ms_per_trajectory": round(traj_ms, 4),
                     "gradient_evals": 21, "ms_per_gradient_eval": round(traj_ms / 21, 5)},
        "hmc": {"transitions": 100, "leapfrog_steps": 20, "step_size": 1e-3,
                "ms_per_transition": round(hmc_ms, 4), "transitions_per_s": round(1e3 / hmc_ms, 2),
                "acceptance": round(hmc_acc, 3), "graph": "10 transitions per replay"},
        "pair_rate_fp64_gpairs_s": round(npairs / (sweep64 * 1e-3) / 1e9, 3),
        "context_paper": "GP100 OpenCL FP64 at N=5338: 4.5 ms likelihood + 4 ms gradient "
                         "(separate evaluations); context only",
    }

    if not args.no_cpu:
        import oracle
        k = max(1, args.cpu_evals)
        t0 = time.perf_counter()
        for _ in range(k):
            ev = oracle.evaluate(prob.x, prob.y, sigma, prob.mask)
        cpu_s = (time.perf_counter() - t0) / k
        out["cpu_baseline"] = {
            "value": round(1.0 / cpu_s, 4), "unit": "evals/s", "cores": 1, "kind": "oracle",
            "sample": f"{k} full fused evaluations of the same N=5392 workload by the serial "
                      "FP64 oracle (one thread)",
            "s_per_eval": round(cpu_s, 4),
        }
        t0 = time.perf_counter()
        k_u = max(1, k // 2)
        for _ in range(k_u):
            oracle.evaluate(prob.x, prob.y, sigma, prob.mask, truncated=False)
        cpu_u = (time.perf_counter() - t0) / k_u
        out["untruncated_model"]["oracle_s_per_eval"] = round(cpu_u, 4)
        out["untruncated_model"]["gpu_over_oracle"] = round(cpu_u / (abl["fp64"]["ms_per_step"] * 1e-3), 1)
        out["untruncated_model"]["truncated_gpu_over_oracle"] = round(cpu_s / (wall64 * 1e-3), 1)
        t0 = time.perf_counter()
        lpd_ref, m_ref = oracle.lpd(xd.cpu().numpy(), [sigma], prob.y, held, prob.mask)
        out["heldout_lpd"]["oracle_s_per_draw"] = round(time.perf_counter() - t0, 4)
        # every accumulated draw is the same state, so the lpd equals the one-draw value
        out["heldout_lpd"]["rel_err_vs_oracle"] = abs(lpd_val - lpd_ref) / abs(lpd_ref)
        g64h = g64.cpu().numpy()
        row64 = np.max(np.abs(g64h - ev.grad), axis=1)
        # the FP32 form against the oracle on the same FP32-rounded Y, per output
        ev32 = oracle.evaluate(prob.x, prob.y.astype(np.float32).astype(np.float64), sigma,
                               prob.mask)
        g32h = P32.unlabel(g32r).cpu().numpy()
        row32 = np.max(np.abs(g32h - ev32.grad), axis=1)
        out["parity"] = {
            "loglik_rel_err_fp64": abs(L64.item() - ev.loglik) / abs(ev.loglik),
            "grad_max_row_err_over_B_fp64": float(np.max(row64 / ev.condrow)),
            "grad_normwise_err_fp64": float(row64.max() / np.abs(ev.grad).max()),
            "dsigma_rel_err_fp64": abs(ds64.item() - ev.dsigma) / abs(ev.dsigma),
            "loglik_rel_err_fp32": abs(L32.item() - ev32.loglik) / abs(ev32.loglik),
            "loglik_rel_err_fp32_vs_fp64_y": abs(L32.item() - ev.loglik) / abs(ev.loglik),
            "grad_max_row_err_over_B_fp32": float(np.max(row32 / ev32.condrow)),
            "grad_max_row_err_over_A_fp32": float(np.max(row32 / np.maximum(ev32.absrow, 1e-300))),
            "grad_normwise_err_fp32": float(row32.max() / np.abs(ev32.grad).max()),
            "dsigma_rel_err_fp32": abs(ds32.item() - ev32.dsigma) / abs(ev32.dsigma),
            "fp32_reference": "oracle on the FP32-rounded Y (arithmetic error); "
                              "loglik_rel_err_fp32_vs_fp64_y includes the rounding of Y",
        }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
