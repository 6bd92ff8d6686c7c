"""Build the CPU oracle (test infrastructure only) with gcc.

Plain C99, -O2, no FMA contraction and no fast-math, so every floating-point
operation is the one written in the source.  OpenMP is linked for the opt-in
parallel-for over domains (orc_set_threads); the default is one thread.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "spkmc_oracle.c")
LIB = os.path.join(HERE, "liboracle_spkmc.so")


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-O2", "-std=c99", "-Wall", "-Wextra", "-fPIC", "-shared",
           "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-o", LIB + ".tmp", SRC, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
