"""GPU: a plain C program drives one fused evaluation through the C ABI alone
(hipMalloc'd buffers, mds_prepare_y, mds_gradient; no Python, no torch in
that process), and a held-out predictive density over two draws in one pass
(mds_heldout_count / fill, mds_lpd_accumulate_draws, mds_lpd_finalize), each
checked against the oracle on the same inputs."""
import os
import subprocess

import numpy as np
import pytest

import oracle
from paper_1905_04582_amd import build, synth

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("case", ["n400_d3", "paper_n5392"])
def test_c_program_matches_oracle(tmp_path, case):
    exe = build.NATIVE_BIN
    assert os.path.exists(exe), "build() compiles tests/native/capi_roundtrip"
    # n400_d3: a small problem; paper_n5392: the paper-scale workload with the
    # default tiling, Y in exact-size device allocations
    p = (synth.make_problem(400, 3, 0.6, seed=77, missing=0.1) if case == "n400_d3"
         else synth.preset("paper_fp64"))
    y = p.y.copy()
    y[p.mask != 0] = np.nan                      # missing pairs travel as NaN
    inp, out = tmp_path / "in.bin", tmp_path / "out.bin"
    with open(inp, "wb") as f:
        np.array([p.n], np.int64).tofile(f)
        np.array([p.d, 0], np.int32).tofile(f)
        np.array([p.sigma], np.float64).tofile(f)
        np.ascontiguousarray(p.x, np.float64).tofile(f)
        np.ascontiguousarray(y, np.float64).tofile(f)
    print(f"native C-ABI run: {case} n={p.n} d={p.d}", flush=True)
    r = subprocess.run([exe, "gpu", str(inp), str(out)], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    raw = np.fromfile(out, np.uint8)
    L, ds = raw[:16].view(np.float64)
    m = int(raw[16:24].view(np.int64)[0])
    g = raw[24:24 + 8 * p.n * p.d].view(np.float64).reshape(p.n, p.d)
    lpd = float(raw[24 + 8 * p.n * p.d:][:8].view(np.float64)[0])
    mh = int(raw[32 + 8 * p.n * p.d:][:8].view(np.int64)[0])
    ref = oracle.evaluate(p.x, p.y, p.sigma, p.mask)
    assert m == ref.m_obs
    assert abs(L - ref.loglik) <= 1e-12 * abs(ref.loglik)
    assert abs(ds - ref.dsigma) <= 1e-12 * ref.abs_dsigma
    assert np.all(np.max(np.abs(g - ref.grad), axis=1) <= 1e-12 * ref.condrow)
    # the held-out density the program computes over two draws in one pass:
    # pairs with (i + j) % 7 == 0, draws x and x + 0.01, sigmas s and 1.1 s
    ii, jj = np.indices((p.n, p.n))
    held = ((ii + jj) % 7 == 0).astype(np.uint8)
    xs = np.stack([p.x, p.x + 0.01])
    lref, mref = oracle.lpd(xs, [p.sigma, 1.1 * p.sigma], y, held)
    assert mh == mref
    assert abs(lpd - lref) <= 1e-12 * abs(lref)
