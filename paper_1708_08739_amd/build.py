"""Build ``libbcd.so`` (HIP, gfx950) next to this file.

Run ``python -m paper_1708_08739_amd.build``.  hipcc cross-compiles for
gfx950 without a GPU present.
"""
from __future__ import annotations

import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libbcd.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

# Packed-FP32 instructions are disabled for all device code.
HIP_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
    "-I", os.path.join(ROOT, "include"),
]


def sources() -> list[str]:
    return sorted(glob.glob(os.path.join(HERE, "csrc", "*.hip")))


GEN_SRC = os.path.join(HERE, "gen", "rmat_draws.c")
GEN_LIB = os.path.join(HERE, "gen", "librmat_draws.so")


def build_gen(verbose: bool = False) -> str:
    """The C form of the input generator's R-MAT draws (host code, gcc)."""
    tmp = GEN_LIB + ".tmp"
    cmd = ["gcc", "-O3", "-fopenmp", "-fPIC", "-shared", "-std=gnu11", "-Wall", "-Wextra",
           "-ffp-contract=off", "-o", tmp, GEN_SRC]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, GEN_LIB)
    return GEN_LIB


def build(verbose: bool = False) -> str:
    build_gen(verbose)
    tmp = LIB + ".tmp"
    cmd = [HIPCC, *HIP_FLAGS, "-o", tmp, *sources(), "-lpthread"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(LIB)
