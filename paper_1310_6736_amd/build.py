"""Builds the gfx950 HIP library libks.so in-tree."""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libks.so")
SOURCES = ["ks_kernels.hip", "ks_abmsod.hip", "ks_runtime.cpp", "ks_server.cpp", "ks_roofline.hip"]

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # decision arithmetic: IEEE double in a fixed order, no contraction into FMA
    "-ffp-contract=off", "-fno-fast-math",
    # no packed fp32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result", "-Wno-unused-value",
]


def build_library(out: str = LIB, verbose: bool = False) -> str:
    srcs = [os.path.join(CSRC, s) for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    cmd = ["/opt/rocm/bin/hipcc", *HIPCC_FLAGS, "-I" + CSRC, "-o", out + ".tmp", *srcs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


if __name__ == "__main__":
    print(build_library(verbose=True))
