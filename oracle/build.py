"""Build the CPU oracle (test infrastructure) as oracle/libvlct_ref.so.

Plain FP64 C: -O2, no fast-math, no FMA contraction, OpenMP over z-planes."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libvlct_ref.so")


def build(verbose: bool = False) -> str:
    src = os.path.join(HERE, "vlct_ref.c")
    cmd = ["gcc", "-std=c11", "-O2", "-fno-fast-math", "-ffp-contract=off", "-fopenmp",
           "-fPIC", "-shared", "-Wall", "-Wextra", "-o", LIB + ".tmp", src, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
