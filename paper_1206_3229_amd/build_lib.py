"""Compile the HIP library for gfx950 (in-tree, no JIT cache).

    python -m paper_1206_3229_amd.build_lib
"""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
SRC = [os.path.join(PKG, "csrc", "vlasov.hip"), os.path.join(PKG, "csrc", "vlasov_batch.hip")]
DEPS = SRC + [os.path.join(PKG, "csrc", n) for n in ("vlasov_kernels.hpp", "vlasov_internal.hpp")] + \
    [os.path.join(ROOT, "include", "vlasov.h")]
LIB = os.path.join(PKG, "libvlasov.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    # IEEE arithmetic exactly as written: no contraction into FMA, no fast math.
    "-ffp-contract=off",
    "-fno-fast-math",
    # no packed FP32 instructions in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall",
    "-Wno-unused-command-line-argument",
    "-Wno-unused-function",
    "-I" + os.path.join(ROOT, "include"),
]


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp"
    cmd = [HIPCC, *FLAGS, *SRC, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


def stale() -> bool:
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    return any(os.path.getmtime(p) > t for p in DEPS)


if __name__ == "__main__":
    print(build(verbose=True))
    sys.exit(0)
