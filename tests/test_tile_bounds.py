"""The pair sweep's tile and wave arithmetic replayed on the host (no GPU):
tests/native/tile_bounds.cpp includes the library's tiling header and calls
the functions the kernel calls (tile_coords, wave_rows) for N = 1..600, 777,
1000, 1536, 5000, 5392, 7999, 20000 and 100000, every valid tiling (rows per
tile, column waves, row waves) and the staging batch of every D.  It checks
that every Y and x row a wave reads, its four-row Y prefetch included, lies
inside the wave's tile and the matrix; that its staging batches cover its
rows in order; that every lower-triangle pair is visited exactly once; and
that every partial-sum slot lies inside its buffer.  Built with
AddressSanitizer and UndefinedBehaviorSanitizer."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")


def test_sweep_rows_and_pairs_in_bounds(tmp_path):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path / "tile_bounds")
    build = subprocess.run(
        [gxx, "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined",
         "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-Wall",
         "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROCM, "include"),
         os.path.join(ROOT, "tests", "native", "tile_bounds.cpp"), "-o", exe],
        capture_output=True, text=True)
    if build.returncode != 0 and "sanitize" in build.stderr:
        pytest.skip("this g++ cannot build sanitized programs: " + build.stderr[-300:])
    assert build.returncode == 0, build.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    run = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert run.returncode == 0, run.stdout + run.stderr
    assert "tile bounds ok" in run.stdout
