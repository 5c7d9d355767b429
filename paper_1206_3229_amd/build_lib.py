"""Compile the HIP library for gfx950 (in-tree, no JIT cache).

Every translation unit under csrc/ is compiled on its own (in parallel), then
linked into libvlasov.so.

    python -m paper_1206_3229_amd.build_lib
"""
from __future__ import annotations

import glob
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
SRC = sorted(glob.glob(os.path.join(CSRC, "*.hip")))
DEPS = SRC + sorted(glob.glob(os.path.join(CSRC, "*.hpp"))) + [os.path.join(ROOT, "include", "vlasov.h")]
LIB = os.path.join(PKG, "libvlasov.so")
OBJDIR = os.path.join(PKG, "_build")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
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


def _jobs() -> int:
    return max(1, min(len(SRC), int(os.environ.get("MAX_JOBS", os.cpu_count() or 1)), 16))


def _compile(src: str, verbose: bool) -> str:
    obj = os.path.join(OBJDIR, os.path.basename(src)[:-4] + ".o")
    cmd = [HIPCC, *FLAGS, "-c", src, "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(OBJDIR, exist_ok=True)
    with ThreadPoolExecutor(_jobs()) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose), SRC))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp]
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
    print(build(verbose="-v" in sys.argv))
    sys.exit(0)
