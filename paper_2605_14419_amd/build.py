"""Builds the HIP library (gfx950) in-tree: paper_2605_14419_amd/_lib/libzsort.so."""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIBDIR = os.path.join(HERE, "_lib")
LIB = os.path.join(LIBDIR, "libzsort.so")
SOURCES = [os.path.join(CSRC, "zsort_kernels.hip"), os.path.join(CSRC, "zsort_learned.hip"),
           os.path.join(CSRC, "zsort_wide.hip"),
           os.path.join(CSRC, "zsort_api.cpp")]

HIPCC_FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-ffp-contract=off",          # every FP64 op of the statistics rounds on its own
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"),
    "-I", CSRC,
]


def build(verbose: bool = False) -> str:
    """Compile every HIP source for gfx950 and link the shared library."""
    os.makedirs(LIBDIR, exist_ok=True)
    tmp = LIB + ".tmp"
    cmd = ["hipcc", *HIPCC_FLAGS, "-shared", "-o", tmp, "-x", "hip", *SOURCES]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
