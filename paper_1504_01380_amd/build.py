"""Build libswept.so (HIP, gfx950) in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
SRC = os.path.join(PKG, "csrc", "swept.hip")
DEPS = [os.path.join(PKG, "csrc", f) for f in ("stencils.hpp", "kernels.hpp")] + \
    [os.path.join(ROOT, "include", h) for h in ("swept.h", "swept_debug.h")]
LIB = os.path.join(PKG, "libswept.so")
LIB_COUNT = os.path.join(PKG, "libswept_count.so")
ARCH = os.environ.get("SWEPT_OFFLOAD_ARCH", "gfx950")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
# roctx ranges around the entry points (rocprofv3 --marker-trace)
LINK = ["-L" + os.path.join(ROCM, "lib"), "-lrocprofiler-sdk-roctx",
        "-Wl,-rpath," + os.path.join(ROCM, "lib")]

# -ffp-contract=off: no fused multiply-add, so every schedule gives the
# oracle's bits.  Packed FP32 instructions are disabled for all device code.
HIPCC_FLAGS = [
    "--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-shared",
    "-ffp-contract=off", "-fno-fast-math",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-command-line-argument",
]


def _compile(out: str, extra, verbose: bool) -> str:
    tmp = out + ".tmp%d" % os.getpid()
    cmd = ["hipcc", *HIPCC_FLAGS, *extra, "-I", os.path.join(ROOT, "include"),
           "-I", os.path.join(PKG, "csrc"), SRC, "-o", tmp, *LINK]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, out)
    return out


def build(verbose: bool = False, counting: bool = True) -> str:
    """Compile csrc/swept.hip into libswept.so next to this file and, with
    counting, the test build libswept_count.so (SWEPT_COUNT_UPDATES: the
    stage kernels count their point updates)."""
    _compile(LIB, [], verbose)
    if counting:
        _compile(LIB_COUNT, ["-DSWEPT_COUNT_UPDATES"], verbose)
    return LIB


def stale() -> bool:
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    return any(os.path.getmtime(p) > t for p in [SRC, *DEPS])


if __name__ == "__main__":
    print(build(verbose=True))
