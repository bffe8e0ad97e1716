"""The C-ABI's host code under AddressSanitizer and UndefinedBehaviorSanitizer
(no GPU).  csrc/mds_api.hip -- argument validation, tiling resolution,
workspace and batch layout, error messages -- is compiled with both
sanitizers on its host side (its device side, the static scratch array, is
unchanged) and linked
with the library's kernel objects into tests/native/capi_sanitize.cpp, which
calls every entry point over a grid of valid and invalid arguments, only
along paths that return before any HIP call.  No report, every expectation
met."""
import os
import shutil
import subprocess

import pytest

from paper_1905_04582_amd import build as hipbuild

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
CSRC = os.path.join(ROOT, "paper_1905_04582_amd", "csrc")
SAN_HOST = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, " ".join(cmd) + "\n" + r.stderr[-3000:]


def test_capi_host_code_clean_under_asan_ubsan(tmp_path):
    clangxx = os.path.join(ROCM, "llvm", "bin", "clang++")
    if not os.path.exists(clangxx) or shutil.which(hipbuild.hipcc()) is None:
        pytest.skip("ROCm clang++/hipcc not available")
    flags = ["-O1", "-g", "-std=c++17", "-fPIC", f"--offload-arch={hipbuild.ARCH}",
             "-I", os.path.join(ROOT, "include")]
    api_o = str(tmp_path / "mds_api_san.o")
    _run([hipbuild.hipcc(), *flags, *SAN_HOST, "-c",
          os.path.join(CSRC, "mds_api.hip"), "-o", api_o])
    # the kernel translation units, unsanitized, as build() compiles them
    objs = []
    for src in hipbuild.SOURCES:
        if src == "mds_api.hip":
            continue
        o = os.path.join(hipbuild.BUILD, os.path.splitext(src)[0] + ".o")
        if not os.path.exists(o) or os.path.getmtime(o) < os.path.getmtime(os.path.join(CSRC, src)):
            o = str(tmp_path / (os.path.splitext(src)[0] + ".o"))
            _run([hipbuild.hipcc(), *hipbuild.common_flags(), "-c", os.path.join(CSRC, src),
                  "-o", o])
        objs.append(o)
    drv_o = str(tmp_path / "drv.o")
    _run([clangxx, "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined",
          "-fno-sanitize-recover=all", "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROCM, "include"),
          "-I", os.path.join(ROOT, "include"), "-c",
          os.path.join(ROOT, "tests", "native", "capi_sanitize.cpp"), "-o", drv_o])
    exe = str(tmp_path / "capi_sanitize")
    _run([clangxx, "-fsanitize=address,undefined", drv_o, api_o, *objs, "-L",
          os.path.join(ROCM, "lib"), "-lamdhip64", f"-Wl,-rpath,{os.path.join(ROCM, 'lib')}",
          "-o", exe])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    run = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert run.returncode == 0, run.stdout + run.stderr
    assert "capi host code ok" in run.stdout
