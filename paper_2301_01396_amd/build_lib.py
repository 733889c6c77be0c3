"""Build ``libxpbd.so`` (HIP, gfx950) in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libxpbd.so")
SOURCES = [os.path.join(CSRC, "xpbd.hip")]
HEADERS = [os.path.join(CSRC, f) for f in sorted(os.listdir(CSRC)) if f.endswith(".hpp")] + [
    os.path.join(os.path.dirname(HERE), "include", "xpbd.h")]

# -O3 without fast-math: IEEE division and square root; multiply-adds are
# fused per source expression only (-ffp-contract=on), so every kernel that
# shares a projection routine rounds it the same way.  Packed-FP32 ops are
# disabled (-packed-fp32-ops) for the device code.
FLAGS = ["-O3", "-std=c++17", "-fPIC", "-shared", "--offload-arch=gfx950", "-ffp-contract=on",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-function", "-L/opt/rocm/lib", "-lrocprofiler-sdk-roctx",
         "-Wl,-rpath,/opt/rocm/lib"]


def build(verbose: bool = False) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tmp = LIB + ".tmp"
    cmd = [hipcc] + FLAGS + ["-o", tmp] + SOURCES
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


def is_stale() -> bool:
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    return any(os.path.getmtime(s) > t for s in SOURCES + HEADERS)


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
