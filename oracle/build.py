"""Build the oracle's shared library (plain C, FP64, no FMA contraction, no fast-math).

Test infrastructure: the oracle is the independent CPU reference for the
immersed-boundary step.  ``python oracle/build.py`` writes ``oracle/libibo_oracle.so``.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libibo_oracle.so")


def build(verbose: bool = False) -> str:
    src = os.path.join(HERE, "ibo.c")
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-std=c99",
           "-Wall", "-shared", "-fPIC", "-o", tmp, src, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
