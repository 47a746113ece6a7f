"""Build the FP64 oracle shared library (test infrastructure only).

Compiled with gcc at -O2 with floating-point contraction disabled, so every
product and sum is rounded separately as written in the C source.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "ibmg_oracle.c")
LIB = os.path.join(HERE, "libibmg_oracle.so")


def build(verbose=False):
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c11", "-D_GNU_SOURCE",
           "-Wall", "-Wno-unused-function", "-fPIC", "-shared", "-o", LIB, SRC, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    return LIB


def ensure_built():
    if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        build()
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
