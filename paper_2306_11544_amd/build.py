"""Builds libmech.so (the HIP kernels and C ABI: the mechanics step and the
microenvironment solver) in-tree for gfx950 with hipcc."""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(HERE, "csrc", "mech.hip")
SOURCES = [SRC, os.path.join(HERE, "csrc", "microenv.hip")]
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libmech.so")

HIP_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # keep packed FP32 instructions out of the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found: the HIP toolchain (ROCm) is required to build libmech.so")


def build(verbose: bool = False, extra=()) -> str:
    """Compile csrc/*.hip into paper_2306_11544_amd/libmech.so (always recompiles)."""
    tmp = LIB + ".tmp"
    cmd = [hipcc(), *HIP_FLAGS, *extra, "-I", INCLUDE, *SOURCES, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError(f"hipcc failed building {' '.join(SOURCES)}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
