"""Build the gfx950 HIP library libvlct.so in-tree with hipcc."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libvlct.so")
SOURCES = [os.path.join(HERE, "csrc", "vlct.hip"), os.path.join(HERE, "csrc", "vlct_adjoint.hip")]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
         # no packed-FP32 instructions in any generated code
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         # FP64 division as the hardware reciprocal with two Newton steps and
         # one residual correction, without the scaling and fix-up steps for
         # subnormal and overflowing quotients (8 instructions instead of 11;
         # bitwise the same results on the turbulence workloads)
         "-fapprox-func"]


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp"
    cmd = [HIPCC] + FLAGS + ["-o", tmp] + SOURCES
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
