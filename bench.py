"""Benchmark of the VL+CT MHD step on one MI355X.

A step is one pass of the whole hot path (PCM+HLLD predictor, CT, half
update, PLMC/PPMC+HLLD corrector, CT, full update, CFL reduction) over the
synthetic workload, with the state resident in HBM and dt chained on the
device.  Prints ONE JSON line with the whole-job throughput, the roofline of
the dominant kernel (timed live with HIP events on the stream it is launched
on) and a CPU baseline (the oracle on a bounded sample of the same workload).

    python bench.py [--steps K] [--warmup W] [--workload NAME] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import ctypes
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Algorithmic FP64 operations per face of the corrector flux kernel (one
# reconstruction -- each cell serves its two faces -- and one HLLD solve), counted by
# paper_2402_05240_amd/csrc/flop_count.cpp
# (add/sub/mul/div/sqrt = 1 FLOP each; mean over turbulence-like states).
FLOPS_PER_FACE = {2: 662.0, 3: 1034.0, 1: 291.0}
# MI355X FP64 vector peak: 256 CUs x 4 SIMDs x 16 lanes x 2 (FMA) x 2.4 GHz.
PEAK_FP64_TFLOPS = 78.6
PEAK_HBM_GBS = 8000.0

WORKLOADS = {
    # name -> (constructor args, metric label)
    "turbulence_plmc_256": dict(kind="turbulence", n=256, recon=2),
    "turbulence_ppmc_256": dict(kind="turbulence", n=256, recon=3),
    "blast_ppmc_512": dict(kind="blast", n=512, recon=3),
    "linear_fast_32": dict(kind="linear", n=32, recon=2),
}


class HipEvents:
    """hipEventCreate / hipEventRecord / hipEventElapsedTime through ctypes."""

    def __init__(self):
        self.hip = ctypes.CDLL("libamdhip64.so")
        self.hip.hipEventCreate.argtypes = [ctypes.POINTER(ctypes.c_void_p)]
        self.hip.hipEventRecord.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
        self.hip.hipEventElapsedTime.argtypes = [ctypes.POINTER(ctypes.c_float), ctypes.c_void_p,
                                                 ctypes.c_void_p]
        self.hip.hipEventSynchronize.argtypes = [ctypes.c_void_p]
        self.hip.hipEventDestroy.argtypes = [ctypes.c_void_p]
        self.pool = []

    def new(self):
        if self.pool:
            return self.pool.pop()
        ev = ctypes.c_void_p()
        rc = self.hip.hipEventCreate(ctypes.byref(ev))
        if rc != 0:
            raise RuntimeError("hipEventCreate failed (%d)" % rc)
        return ev.value

    def record(self, ev, stream):
        rc = self.hip.hipEventRecord(ctypes.c_void_p(ev), ctypes.c_void_p(stream))
        if rc != 0:
            raise RuntimeError("hipEventRecord failed (%d)" % rc)

    def elapsed_ms(self, a, b):
        self.hip.hipEventSynchronize(ctypes.c_void_p(b))
        ms = ctypes.c_float()
        rc = self.hip.hipEventElapsedTime(ctypes.byref(ms), ctypes.c_void_p(a), ctypes.c_void_p(b))
        if rc != 0:
            raise RuntimeError("hipEventElapsedTime failed (%d)" % rc)
        return float(ms.value)

    def release(self, ev):
        self.pool.append(ev)


class KernelTimer:
    """Brackets every launch of each kernel family with HIP events on the
    stream the library launches it on (via the library's launch observer)."""

    def __init__(self, vlct, events: HipEvents):
        self.vlct = vlct
        self.ev = events
        self.active = False
        self.open = {}
        self.pairs = {}

    def __call__(self, kernel, phase, stream):
        if not self.active:
            return
        if phase == 0:
            e = self.ev.new()
            self.ev.record(e, stream)
            self.open[kernel] = e
        else:
            e = self.ev.new()
            self.ev.record(e, stream)
            self.pairs.setdefault(kernel, []).append((self.open.pop(kernel), e))

    def summary(self):
        out = {}
        for k, pairs in self.pairs.items():
            ms = [self.ev.elapsed_ms(a, b) for a, b in pairs]
            out[self.vlct.vlct_kernel_name(k)] = {"launches": len(ms), "total_ms": sum(ms),
                                                  "avg_ms": sum(ms) / len(ms)}
        return out


def make_workload(name):
    from paper_2402_05240_amd import inputs as I
    w = WORKLOADS[name]
    n = w["n"]
    if w["kind"] == "turbulence":
        g, s = I.turbulence((n, n, n), recon=w["recon"])
    elif w["kind"] == "blast":
        g, s = I.blast((n, n, n), b0=1.0, recon=w["recon"])
    else:
        g, s, _ = I.linear_wave((n, n, n), "fast", recon=w["recon"])
    return g, s


def cpu_baseline(g, s, planes: int, threads: int):
    """One oracle step on a z-slab of the workload's own initial state."""
    import numpy as np
    from oracle import build as refbuild
    from oracle import ref
    from paper_2402_05240_amd import inputs as I
    if not os.path.exists(ref.LIB_PATH):
        refbuild.build()
    planes = min(planes, g.nz)
    sg = I.Grid(g.nx, g.ny, planes, g.dx, g.dy, g.dz, g.gamma, g.cfl, g.recon, g.bc)
    ss = {f: np.ascontiguousarray(s[f][: planes + (1 if f == "bz" else 0)]) for f in I.FIELDS}
    if g.bc[2] == I.BC_PERIODIC:
        ss["bz"][-1] = ss["bz"][0]
    dt = ref.cfl_dt(sg, ss, threads)
    t0 = time.perf_counter()
    ref.step(sg, ss, dt, nthreads=threads)
    sec = time.perf_counter() - t0
    cells = sg.ncells
    return {"value": cells / sec, "unit": "cell updates/s", "cores": threads, "kind": "oracle",
            "sample": "one oracle step (predictor+corrector+dt) on a %dx%dx%d z-slab of the "
                      "workload's initial state, %.1f s on %d host threads" % (
                          g.nx, g.ny, planes, sec, threads)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="turbulence_plmc_256", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-planes", type=int, default=32)
    ap.add_argument("--cpu-threads", type=int, default=0)
    ap.add_argument("--copy-calibration-gib", type=float, default=0.0,
                    help="first run one device-to-device copy of this many GiB (a plain copy "
                         "kernel of known size, to calibrate HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on exactly one GPU: this build has no multi-GPU path "
              "(requested --gpus %d)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2402_05240_amd import vlct
    from paper_2402_05240_amd.device import Stepper

    if args.copy_calibration_gib > 0:
        nbytes = int(args.copy_calibration_gib * (1 << 30))
        src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        torch.cuda.empty_cache()
        print("copy calibration: %d bytes read and written" % nbytes, file=sys.stderr)

    g, s0 = make_workload(args.workload)
    st = Stepper(g, device="cuda:0").upload(s0)
    stream = torch.cuda.current_stream()
    st.compute_dt()
    for _ in range(args.warmup):
        st.step()
    torch.cuda.synchronize()

    events = HipEvents()
    timer = KernelTimer(vlct, events)
    vlct.vlct_set_launch_observer(timer)
    e0, e1 = events.new(), events.new()
    torch.cuda.synchronize()
    timer.active = True
    w0 = time.perf_counter()
    events.record(e0, stream.cuda_stream)
    for _ in range(args.steps):
        st.step()
    events.record(e1, stream.cuda_stream)
    torch.cuda.synchronize()
    w1 = time.perf_counter()
    timer.active = False
    vlct.vlct_set_launch_observer(None)
    ms_total = events.elapsed_ms(e0, e1)
    kern = timer.summary()
    status = st.status_bits()

    ncell = g.ncells
    ms_step = ms_total / args.steps
    value = ncell * args.steps / (ms_total * 1e-3)
    dom = kern.get("flux_recon_hlld")
    faces_per_launch = ncell              # one axis' faces of a periodic grid
    flops_launch = FLOPS_PER_FACE[g.recon] * faces_per_launch
    achieved = flops_launch / (dom["avg_ms"] * 1e-3) / 1e12
    recon_name = {1: "PCM", 2: "PLMC", 3: "PPMC"}[g.recon]
    out = {
        "metric": "FP64 cell updates/s (PLMC+HLLD, 256^3)",
        "value": value,
        "unit": "cell updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "grid": [g.nx, g.ny, g.nz],
                   "reconstruction": recon_name, "riemann": "HLLD", "integrator": "VL+CT",
                   "bc": ["periodic" if b == 0 else "outflow" for b in g.bc], "cfl": g.cfl,
                   "gamma": g.gamma},
        "roofline": {"bound": "alu", "kernel": "flux_recon_hlld", "achieved": achieved,
                     "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP64_TFLOPS, "traffic": None,
                     "flops_per_launch": flops_launch, "avg_launch_ms": dom["avg_ms"]},
        "kernels_ms_per_step": {k: v["total_ms"] / args.steps for k, v in kern.items()},
        "wall_ms_per_step": (w1 - w0) * 1e3 / args.steps,
        "status": status,
    }
    if not args.no_cpu_baseline:
        del st
        torch.cuda.empty_cache()
        threads = args.cpu_threads or min(16, os.cpu_count() or 1)
        out["cpu_baseline"] = cpu_baseline(g, s0, args.cpu_planes, threads)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
