"""Build the FP64 CPU oracle (test infrastructure) as a shared library with gcc.

The oracle is never linked into the product library; this script only compiles
``pdhg_oracle.c`` next to itself.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "pdhg_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")


def build(verbose: bool = False) -> str:
    # -ffp-contract=off keeps every product and sum separately rounded, so that
    # exact-scaling tests see IEEE arithmetic exactly as written.
    cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
           "-ffp-contract=off", "-o", LIB, SRC, "-lm"]
    if verbose:
        print(" ".join(cmd), file=sys.stderr)
    subprocess.run(cmd, check=True)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
