"""Compile the C oracle into ``oracle/libddgs_oracle.so`` with gcc.

Plain IEEE double arithmetic: no fast-math and no floating-point
contraction, so every expression is evaluated as written.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "ddgs_oracle.c")
LIB = os.path.join(HERE, "libddgs_oracle.so")


def build(verbose=False):
    cmd = ["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-fPIC", "-shared", "-fopenmp",
           "-ffp-contract=off", "-fno-fast-math", "-march=x86-64-v2",
           "-Wall", "-Wextra", "-Wno-unused-parameter",
           SRC, "-o", LIB + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


def ensure_built():
    if not os.path.exists(LIB) or os.path.getmtime(LIB) < max(
            os.path.getmtime(SRC), os.path.getmtime(os.path.join(HERE, "ddgs_oracle.h"))):
        build()
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
