"""Builds the oracle's C library (test infrastructure only).

The flags keep the arithmetic plain: no fused multiply-add contraction and
the textbook complex product.  The code is generic x86-64, so the library
also runs on a host whose CPU differs from the build machine's.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "eigh.c")
LIB = os.path.join(HERE, "liboracle.so")
CFLAGS = ["-O3", "-std=c11", "-fPIC", "-shared", "-fopenmp",
          "-ffp-contract=off", "-fcx-limited-range"]


def build(verbose: bool = False) -> str:
    cmd = ["gcc", *CFLAGS, SRC, "-o", LIB + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
