"""Build libmassivemds.so (HIP, gfx950) in-tree with hipcc.

    python -m paper_1905_04582_amd.build [-DMACRO=value ...] [--out other.so]

Every translation unit under csrc/ is compiled for gfx950 only, with packed
FP32 instructions disabled and no implicit multiply-add contraction, then
linked into paper_1905_04582_amd/libmassivemds.so.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libmassivemds.so")
SOURCES = ["mds_api.hip", "mds_kernels.hip", "mds_order.hip", "mds_hmc.hip", "mds_lpd.hip",
           "mds_sweep_f64.hip", "mds_sweep_f32.hip"]
ARCH = "gfx950"


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found: the MI355X library cannot be built")


def common_flags():
    return ["-O3", "-std=c++17", "-fPIC", "-fvisibility=hidden", f"--offload-arch={ARCH}",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            # no implicit multiply-add fusion: every fused operation is an
            # explicit fma(), so each kernel instantiation (with or without
            # the gradient, single or batched) rounds the same expressions the
            # same way
            "-ffp-contract=off",
            "-Wall", "-Wno-unused-result", "-I", os.path.join(ROOT, "include")]


def _compile(src: str, extra, tag: str = "") -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + tag + ".o")
    cmd = [hipcc(), *common_flags(), *extra, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{r.stderr}")
    return obj


def build(extra_flags=(), verbose: bool = False, out: str | None = None) -> str:
    """Compile and link; `out` (default: the in-package library) names the .so."""
    os.makedirs(BUILD, exist_ok=True)
    lib = out or LIB
    tag = "" if out is None else "_" + os.path.splitext(os.path.basename(out))[0]
    jobs = min(len(SOURCES), max(1, (os.cpu_count() or 4)))
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, list(extra_flags), tag), SOURCES))
    tmp = lib + ".tmp%d" % os.getpid()
    cmd = [hipcc(), "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, lib)
    if verbose:
        print("built", lib)
    return lib


NATIVE_SRC = os.path.join(ROOT, "tests", "native", "capi_roundtrip.c")
NATIVE_BIN = os.path.join(ROOT, "tests", "native", "capi_roundtrip")


def build_native_check(out: str = NATIVE_BIN) -> str:
    """Compile the plain C program that drives the library through its C ABI
    alone (host C compiler; links libmassivemds and the HIP runtime)."""
    cc = shutil.which("gcc") or shutil.which("cc")
    if not cc:
        raise RuntimeError("no C compiler for the native C-ABI check")
    rocm = os.path.dirname(os.path.dirname(hipcc()))
    cmd = [cc, "-std=c11", "-O2", "-Wall", "-D__HIP_PLATFORM_AMD__",
           "-I", os.path.join(rocm, "include"), "-I", os.path.join(ROOT, "include"),
           NATIVE_SRC, "-o", out, "-L", PKG, "-lmassivemds", "-L", os.path.join(rocm, "lib"),
           "-lamdhip64", f"-Wl,-rpath,{PKG}", f"-Wl,-rpath,{os.path.join(rocm, 'lib')}"]
    if os.path.abspath(out) == NATIVE_BIN:
        # the in-tree program finds the library next to it wherever the tree is copied
        cmd.insert(-3, "-Wl,-rpath,$ORIGIN/../../paper_1905_04582_amd")
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"native C-ABI check failed to build:\n{r.stderr}")
    return out


if __name__ == "__main__":
    # python -m paper_1905_04582_amd.build [-DMACRO=value ...] [--out path/to/lib.so]
    argv = sys.argv[1:]
    out = None
    if "--out" in argv:
        k = argv.index("--out")
        out = os.path.abspath(argv[k + 1])
        argv = argv[:k] + argv[k + 2:]
    build(argv, verbose=True, out=out)
