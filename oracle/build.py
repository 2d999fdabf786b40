"""Builds the CPU oracle (test infrastructure) into oracle/libtsdf_oracle.so.

The flags keep every binary32 operation a single correctly rounded IEEE-754
operation: no contraction into fused multiply-add, no fast-math, SSE scalar
arithmetic (the x86-64 default).  OpenMP serves only the multi-threaded
entry point used to time the CPU baseline on all cores.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libtsdf_oracle.so")
CFLAGS = ["-std=c99", "-O2", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math",
          "-fexcess-precision=standard", "-fopenmp", "-Wall", "-Wno-unused-function"]


def build(verbose: bool = False) -> str:
    src = os.path.join(HERE, "tsdf_oracle.c")
    tmp = LIB + ".tmp"
    cmd = ["gcc", *CFLAGS, "-o", tmp, src, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True, cwd=HERE)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
