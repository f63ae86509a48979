"""Builds the FP64 oracle library (oracle/libpfo.so) with gcc.

Flags: -O2 -ffp-contract=off (no fused multiply-add contraction), no
fast-math, so the library evaluates every expression as written in IEEE
binary64 with round-to-nearest-even; -fopenmp splits the per-node loops over
rows (the arithmetic of each node does not depend on the thread count).
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libpfo.so")


def build(verbose: bool = False) -> str:
    src = os.path.join(HERE, "pfo.c")
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c11", "-Wall", "-Wextra",
           "-fopenmp", "-fPIC", "-shared", src, "-o", LIB + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
