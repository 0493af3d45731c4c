"""Compile the oracle's C code into oracle/liboracle.so (gcc + OpenMP).

Test infrastructure: building the checker is not using it.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "direct.c")
LIB = os.path.join(HERE, "liboracle.so")

# Portable x86-64 baseline (the library may run on another host than it was
# built on); no FMA contraction so the arithmetic is the plain written one.
CFLAGS = ["-O3", "-march=x86-64-v2", "-fopenmp", "-ffp-contract=off",
          "-fno-fast-math", "-shared", "-fPIC", "-std=c11"]


def build(verbose=False):
    tmp = LIB + ".tmp"
    cmd = ["gcc", *CFLAGS, SRC, "-o", tmp, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
