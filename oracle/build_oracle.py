"""Compile the oracle's C direct sum (test infrastructure only).

    python oracle/build_oracle.py

writes oracle/liboracle_direct.so with gcc -O2 -fopenmp.  No fast-math flags:
the oracle keeps IEEE FP64 semantics.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "direct_sum.c")
LIB = os.path.join(HERE, "liboracle_direct.so")


def build(verbose=False):
    cmd = ["gcc", "-O2", "-fPIC", "-shared", "-fopenmp", "-std=c11",
           "-D_DEFAULT_SOURCE", SRC, "-o", LIB + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
