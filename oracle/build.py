"""Build the CPU oracle shared library (test infrastructure only).

    python oracle/build.py

Compiles m2s_oracle.c with gcc -O2 -ffp-contract=off (no FMA contraction,
no fast-math, single-threaded) into oracle/libm2s_oracle.so.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libm2s_oracle.so")


def build(verbose: bool = False) -> str:
    src = os.path.join(HERE, "m2s_oracle.c")
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-std=c11", "-O2", "-ffp-contract=off", "-fno-fast-math",
           "-fPIC", "-shared", "-Wall", "-Wextra", "-Wno-unused-function",
           "-o", tmp, src, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
