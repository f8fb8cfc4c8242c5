"""Builds the HIP library (gfx950) in-tree: paper_2609_34935_amd/libqram_hip.so."""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRCS = [os.path.join(HERE, "csrc", f) for f in ("qram_host.hip", "qram_kernels.hip", "qram_evolve.hip", "qram_plain.hip", "qram_server.hip", "qram_dense.hip")]
LIB = os.path.join(HERE, "libqram_hip.so")

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # no packed fp32 instructions in any generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # the register-held site lists index their entries with unrolled loops
    # only; a partial unroll would move them to scratch memory
    "-mllvm", "-pragma-unroll-threshold=200000",
]


def build_library(verbose: bool = False) -> str:
    """Compile every HIP source of the package into one shared library."""
    hipcc = os.environ.get("HIPCC", "hipcc")
    tmp = LIB + ".tmp"
    cmd = [hipcc, *HIPCC_FLAGS, "-o", tmp, *SRCS]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build_library(verbose=True))
