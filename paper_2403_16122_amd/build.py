"""Build the gfx950 shared library ``liblbm.so`` in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "liblbm.so")
SOURCES = [os.path.join(CSRC, f) for f in ("lbm_kernels.hip", "lbm_api.hip", "lbm_batch.hip", "lbm_mlp.hip")]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

# Packed-FP32 instructions are disabled for all device code (they have been
# observed to give wrong results on these parts); -O3 otherwise free to
# contract into FMAs.
FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "-shared", "--offload-arch=gfx950",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def build_library(extra_flags=None, verbose: bool = False) -> str:
    cmd = [HIPCC] + FLAGS + list(extra_flags or []) + [
        "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-o", LIB + ".tmp"] + SOURCES
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build_library(sys.argv[1:], verbose=True)
