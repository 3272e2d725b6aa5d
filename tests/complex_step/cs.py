"""Complex-step derivatives of the CPU oracle's steps (test infrastructure).

build(tmpdir) compiles tests/complex_step/cs_oracle.cpp -- the unchanged
oracle source compiled with a complex-step scalar -- into a shared library;
jvp(g, s, ds, dts) returns (state after the steps, J ds) for a perturbation
direction ds, with J the Jacobian of the steps at s (step sizes fixed)."""
import ctypes
import os
import shutil
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ORACLE = os.path.join(os.path.dirname(os.path.dirname(HERE)), "oracle")
FIELDS = ("rho", "mx", "my", "mz", "E", "bx", "by", "bz")
H = 1e-30  # imaginary step: J ds = Im(out) / H, exact to rounding

_DP = ctypes.POINTER(ctypes.c_double)


class ComplexStepOracle:
    def __init__(self, lib_path):
        self.lib = ctypes.CDLL(lib_path)
        self.lib.cs_run.argtypes = [ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_double),
                                    ctypes.c_double, ctypes.c_double, ctypes.c_int32,
                                    ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(_DP),
                                    ctypes.POINTER(_DP), ctypes.POINTER(ctypes.c_double),
                                    ctypes.c_int, ctypes.POINTER(_DP), ctypes.POINTER(_DP),
                                    ctypes.POINTER(ctypes.c_uint32)]
        self.lib.cs_run.restype = ctypes.c_int

    def jvp(self, g, s, ds, dts):
        re = [np.ascontiguousarray(s[f], dtype=np.float64) for f in FIELDS]
        im = [np.ascontiguousarray(H * ds[f], dtype=np.float64) for f in FIELDS]
        ore = [np.empty_like(x) for x in re]
        oim = [np.empty_like(x) for x in re]

        def ptrs(arrs):
            return (_DP * 8)(*[a.ctypes.data_as(_DP) for a in arrs])
        n = (ctypes.c_int32 * 3)(g.nx, g.ny, g.nz)
        dl = (ctypes.c_double * 3)(g.dx, g.dy, g.dz)
        bc = (ctypes.c_int32 * 3)(*[int(b) for b in g.bc])
        d = (ctypes.c_double * len(dts))(*dts)
        st = ctypes.c_uint32(0)
        rc = self.lib.cs_run(n, dl, float(g.gamma), float(g.cfl), int(g.recon), bc, ptrs(re),
                             ptrs(im), d, len(dts), ptrs(ore), ptrs(oim), ctypes.byref(st))
        if rc != 0:
            raise RuntimeError("complex-step oracle returned %d" % rc)
        out = dict(zip(FIELDS, ore))
        jv = {f: x / H for f, x in zip(FIELDS, oim)}
        return out, jv, st.value


def build(tmpdir) -> ComplexStepOracle:
    gxx = shutil.which("g++")
    if gxx is None:
        raise RuntimeError("no host C++ compiler")
    tmpdir = str(tmpdir)
    shutil.copy(os.path.join(ORACLE, "vlct_ref.c"), os.path.join(tmpdir, "vlct_ref.c"))
    # the oracle's header without its C-linkage block (the scalar type is a class here)
    with open(os.path.join(ORACLE, "vlct_ref.h")) as f:
        lines = f.read().splitlines()
    out, skip = [], 0
    for ln in lines:
        if ln.strip() == "#ifdef __cplusplus":
            skip = 3  # '#ifdef __cplusplus', 'extern "C" {' or '}', '#endif'
        if skip:
            skip -= 1
            continue
        out.append(ln)
    with open(os.path.join(tmpdir, "vlct_ref.h"), "w") as f:
        f.write("\n".join(out) + "\n")
    shutil.copy(os.path.join(HERE, "cs_oracle.cpp"), os.path.join(tmpdir, "cs_oracle.cpp"))
    lib = os.path.join(tmpdir, "libcs_oracle.so")
    subprocess.run([gxx, "-O2", "-std=c++17", "-fpermissive", "-w", "-fPIC", "-shared", "-o", lib,
                    os.path.join(tmpdir, "cs_oracle.cpp")], check=True, cwd=tmpdir)
    return ComplexStepOracle(lib)
