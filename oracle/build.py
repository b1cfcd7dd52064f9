"""Build the CPU oracle shared library (test infrastructure only).

The oracle is plain C compiled with -ffp-contract=off so that every fused
multiply-add in it is an explicit fma() call; -fopenmp for its optional
phase-parallel mode (same results as the serial run).
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "ec_oracle.c")
LIB = os.path.join(HERE, "libec_oracle.so")


FLAGS = ["-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math",
         "-fopenmp", "-Wall", "-Wextra"]


def build(verbose: bool = False) -> str:
    cmd = ["gcc"] + FLAGS + ["-o", LIB + ".tmp", SRC, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
