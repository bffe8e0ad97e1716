"""The C oracle under AddressSanitizer and UndefinedBehaviorSanitizer (host
only): tests/native/oracle_sanitize.c drives every entry point on small
problems (empty, one point, coincident points, masks, NaN entries, padded
leading dimensions) and must finish without a sanitizer report."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_oracle_clean_under_asan_ubsan(tmp_path):
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc not available")
    exe = str(tmp_path / "oracle_sanitize")
    build = subprocess.run(
        [gcc, "-std=c99", "-O1", "-g", "-fsanitize=address,undefined",
         "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-fno-fast-math",
         "-ffp-contract=off", "-Wall", "-Wextra",
         os.path.join(ROOT, "oracle", "mds_oracle.c"),
         os.path.join(ROOT, "tests", "native", "oracle_sanitize.c"), "-lm", "-o", exe],
        capture_output=True, text=True)
    if build.returncode != 0 and "sanitize" in build.stderr:
        pytest.skip("this gcc cannot build sanitized programs: " + build.stderr[-300:])
    assert build.returncode == 0, build.stderr
    # verify_asan_link_order=0: tolerate a library the environment preloads
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    run = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=120)
    assert run.returncode == 0, run.stdout + run.stderr
    assert "ok" in run.stdout
