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
import math
import ctypes
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Algorithmic FP64 operations per unit of the compute-heavy kernel families,
# counted by paper_2402_05240_amd/csrc/flop_count.cpp (add/sub/mul/div/sqrt = 1
# FLOP each, mean over smooth random stencils): a corrector face needs one
# reconstruction (each cell's serves its two faces) and one HLLD solve; a
# predictor cell three PCM HLLD solves plus its primitives, edge fields and
# updates.
FLOPS_PER_FACE = {1: 268.0, 2: 640.0, 3: 1067.0, 4: 359.0, 5: 746.1}
FLOPS_PER_PRED_CELL = 999.0
# MI355X FP64 vector peak: 256 CUs x 4 SIMDs x 16 lanes x 2 (FMA) x 2.4 GHz.
PEAK_FP64_TFLOPS = 78.6
PEAK_HBM_GBS = 8000.0
F64 = 8
# The algorithmic minimum of the whole step (the scope's per-unit figure): read
# U^n and write U^{n+1}, 8 + 8 doubles per cell update.
STEP_MIN_BYTES_PER_CELL = 16 * F64
# Design HBM bytes per unit of each kernel family as written (units: cells,
# ghost cells for the ghost-layer primitive kernel):
#   predictor  reads U^n (5 cell + 3 face fields), writes U^{n+1/2} (8) and
#              the interior half-step primitives (8)
#   prims      (ghost layers) reads 8 fields, writes 8 primitives
#   ct_update  reads 5 cell + 3 face fields of U^n, 3 axes x 7 flux components
#              and the upwind bytes, 6 primitives (v, B_cc for -v x B); writes
#              5 + 3 fields (the CFL maxima of the new state cost no bytes)
#   dt         reads 5 cell + 3 face fields (vlct_cfl_dt and in-place steps)
#   flux_recon_hlld  8 primitives + normal field in, 7 flux components + the
#              upwind byte out, per face
BYTES_PER_UNIT = {"predictor": 24 * F64, "prims": 16 * F64, "ct_update": 43 * F64 + 3,
                  "dt": 8 * F64, "flux_recon_hlld": 16 * F64 + 1, "flux_pcm_hlld": 16 * F64 + 1}
COUNTERS_FILE = os.path.join(ROOT, "profiles", "hbm_counters_turbulence_plmc_256.json")
VALU_FILE = os.path.join(ROOT, "profiles", "fp64_valu_turbulence_plmc_256.json")
SOURCES = ("paper_2402_05240_amd/csrc/vlct.hip", "paper_2402_05240_amd/csrc/vlct_common.hpp",
           "paper_2402_05240_amd/csrc/mhd_physics.hpp", "paper_2402_05240_amd/build.py")


def source_hash():
    """sha256 over the kernel sources and their compiler flags: counter
    figures are valid only for them."""
    import hashlib
    h = hashlib.sha256()
    for rel in SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


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


WORKLOAD_STEPS = {"turbulence_ppmc_256": 20, "blast_ppmc_512": 50, "linear_fast_32": 82}


def workload_bench(name, warmup=3):
    """Cell updates per second of one more workload: its run length (100 steps
    of turbulence are timed as 20, the blast's 50 steps and the linear wave's
    82-step period in full), dt chained on the device, with the bytes per
    cell update the fused minimum implies."""
    import torch
    from paper_2402_05240_amd.device import Stepper
    g, s0 = make_workload(name)
    st = Stepper(g, device="cuda:0").upload(s0)
    st.compute_dt()
    for _ in range(warmup):
        st.step()
    steps = WORKLOAD_STEPS[name]
    st.upload(s0)
    del s0
    st.compute_dt()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(steps):
        st.step()
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / steps
    value = g.ncells / (ms * 1e-3)
    return {"grid": [g.nx, g.ny, g.nz], "reconstruction": RECON_NAMES[g.recon],
            "bc": ["periodic" if x == 0 else "outflow" for x in g.bc], "steps": steps,
            "ms_per_step": ms, "value": value, "unit": "cell updates/s",
            "frac_hbm_min": STEP_MIN_BYTES_PER_CELL * value / (PEAK_HBM_GBS * 1e9),
            "status": st.status_bits()}


def progress(msg):
    """One line on stderr per finished part of the run (the JSON result goes
    to stdout alone)."""
    print("bench: %s" % msg, file=sys.stderr, flush=True)


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


def cpu_baseline(g, s, planes: int, steps: int, threads: int):
    """The oracle, as it stands, on a bounded sample of the workload: `steps`
    steps of a z-slab of `planes` planes of its initial state."""
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
    for _ in range(steps):
        ss, dt, _ = ref.step(sg, ss, dt, nthreads=threads)
    sec = time.perf_counter() - t0
    return {"value": sg.ncells * steps / sec, "unit": "cell updates/s", "cores": threads,
            "kind": "oracle",
            "sample": "%d oracle steps (predictor+corrector+dt, dt chained) on a %dx%dx%d "
                      "slab of the workload's initial state: %.1f s on %d host threads" % (
                          steps, g.nx, g.ny, planes, sec, threads)}


HEADLINE_METRIC = "FP64 cell updates/s (PLMC+HLLD, 256^3); % HBM peak; adjoint/forward cost"


def _load_profile(path, workload):
    """A committed counter summary, when it was taken on this workload with
    these kernel sources (else {})."""
    try:
        with open(path) as f:
            c = json.load(f)
    except (OSError, ValueError):
        return {}
    if c.get("source_sha256") != source_hash() or c.get("workload") != workload:
        return {}
    return c.get("families", {})


def load_traffic(workload):
    """Per-launch HBM bytes of each kernel family (FETCH_SIZE + WRITE_SIZE)."""
    return {k: v["traffic_bytes_per_launch"]
            for k, v in _load_profile(COUNTERS_FILE, workload).items()}


def load_valu(workload):
    """Per-family FP64 VALU counters (instructions per launch, VALU busy)."""
    return _load_profile(VALU_FILE, workload)


def rooflines(g, kern, steps, workload=None):
    """Roofline of every kernel family, from the launches timed with HIP events
    on the library's stream: achieved = algorithmic work per launch / average
    launch duration, against the roof the family's counters say binds it (FP64
    VALU issue when the VALU is busier than HBM is, else HBM bandwidth); with
    no counters for these sources, the design's label."""
    ncell = g.ncells
    nghost = (g.nx + 6) * (g.ny + 6) * (g.nz + 6) - ncell
    traffic = load_traffic(workload) if workload else {}
    valu = load_valu(workload) if workload else {}
    fam = {}
    for name, v in kern.items():
        key = "ct_update" if name in ("update_half", "update_full") else name
        f = fam.setdefault(key, {"launches": 0, "total_ms": 0.0})
        f["launches"] += v["launches"]
        f["total_ms"] += v["total_ms"]
    out = {}
    for key, f in fam.items():
        avg_ms = f["total_ms"] / f["launches"]
        r = {"kernel": key, "launches_per_step": f["launches"] / steps,
             "ms_per_step": f["total_ms"] / steps, "avg_launch_ms": avg_ms}
        if key == "dt_final":
            # one block reducing the CT blocks' CFL maxima: launch latency
            r.update({"bound": "latency", "achieved": None, "peak": None, "unit": None,
                      "frac": None, "per_unit": "the maxima of the full update's blocks",
                      "bytes_per_step": 0.0, "traffic": None})
            out[key] = r
            continue
        units = nghost if key == "prims" else ncell
        nbytes = BYTES_PER_UNIT.get(key, 0) * units
        flops = None
        if key == "flux_recon_hlld":
            flops = FLOPS_PER_FACE[g.recon] * ncell   # one axis' faces per launch
        elif key == "flux_pcm_hlld":
            flops = FLOPS_PER_FACE[1] * ncell
        elif key == "predictor":
            flops = FLOPS_PER_PRED_CELL * ncell
        gbs = nbytes / (avg_ms * 1e-3) / 1e9
        r["hbm_design"] = {"bytes_per_launch": nbytes, "achieved": gbs, "unit": "GB/s",
                           "frac": gbs / PEAK_HBM_GBS,
                           "per_unit": "%d B per %s" % (BYTES_PER_UNIT.get(key, 0),
                                                        "ghost cell" if key == "prims" else
                                                        ("face" if "flux" in key else "cell"))}
        r["bytes_per_step"] = nbytes * f["launches"] / steps
        if flops is not None:
            tf = flops / (avg_ms * 1e-3) / 1e12
            r["fp64_counted"] = {"flops_per_launch": flops, "achieved": tf, "unit": "TFLOP/s",
                                 "frac": tf / PEAK_FP64_TFLOPS}
        tr = traffic.get(key)
        r["traffic"] = tr
        if tr is not None:
            r["traffic_unit"] = "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, calibrated)"
            r["traffic_frac"] = tr / (avg_ms * 1e-3) / 1e9 / PEAK_HBM_GBS
        vc = valu.get(key)
        if vc:
            r["fp64_valu"] = vc
        # the binding roof: from the counters when they exist
        if vc and tr is not None:
            bound = "alu" if vc["valu_busy"] >= r["traffic_frac"] else "hbm"
            r["bound_from"] = "counters (VALU busy %.2f vs HBM traffic %.2f of peak)" % (
                vc["valu_busy"], r["traffic_frac"])
        else:
            bound = "alu" if flops is not None else "hbm"
            r["bound_from"] = "design label (no counters for these sources)"
        if bound == "alu" and flops is not None:
            r.update({"bound": "alu", "achieved": r["fp64_counted"]["achieved"],
                      "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                      "frac": r["fp64_counted"]["frac"],
                      "per_unit": "%.1f FLOP per %s" % (
                          flops / ncell, "cell" if key == "predictor" else "face")})
        else:
            r.update({"bound": "hbm", "achieved": gbs, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                      "frac": gbs / PEAK_HBM_GBS, "per_unit": r["hbm_design"]["per_unit"]})
        out[key] = r
    return out


def step_roofline(rl, value, ncell, design_bytes):
    """Whole-step HBM figures: algorithmic (128 B per cell update), design and
    counted bytes per cell update, each as a fraction of the HBM peak at the
    measured cell-update rate; and the counted FP64 VALU work per cell."""
    out = {"bytes_per_cell_min": STEP_MIN_BYTES_PER_CELL,
           "achieved_min": STEP_MIN_BYTES_PER_CELL * value / 1e9, "unit": "GB/s",
           "frac_min": STEP_MIN_BYTES_PER_CELL * value / (PEAK_HBM_GBS * 1e9),
           "bytes_per_cell_design": design_bytes,
           "frac_design": design_bytes * value / (PEAK_HBM_GBS * 1e9)}
    if all(r.get("traffic") is not None for k, r in rl.items() if k != "dt_final"):
        tb = sum(r["traffic"] * r["launches_per_step"] for k, r in rl.items()
                 if k != "dt_final") / ncell
        out.update({"bytes_per_cell_counters": tb,
                    "frac_counters": tb * value / (PEAK_HBM_GBS * 1e9)})
    flops = [r["fp64_counted"]["flops_per_launch"] * r["launches_per_step"]
             for r in rl.values() if "fp64_counted" in r]
    if flops:
        out["fp64_counted_flops_per_cell"] = sum(flops) / ncell
        out["fp64_counted_frac"] = sum(flops) / ncell * value / (PEAK_FP64_TFLOPS * 1e12)
    return out


def summarize_valu(insts_csv, busy_csv, workload, commands, out_dir):
    """rocprofv3 --pmc runs of FP64 VALU instruction counts (SQ_INSTS_VALU_*_F64,
    SQ_INSTS_VALU, SQ_WAVES) and of VALU busy / utilisation / occupancy
    (VALUBusy, VALUUtilization, MeanOccupancyPerActiveCU) -> per-family means
    per launch (profiles/fp64_valu_<workload>.{json,md}), with the kernels'
    VGPR, LDS and scratch sizes from the same records."""
    import collections
    import csv

    def per_family(path):
        vals = collections.defaultdict(lambda: collections.defaultdict(list))
        res = {}
        for r in csv.DictReader(open(path)):
            k = kernel_family(r["Kernel_Name"])
            if not k or k == "copy":
                continue
            vals[k][r["Counter_Name"]].append(float(r["Counter_Value"]))
            res.setdefault(k, set()).add((r["Kernel_Name"].split("(")[0].replace("void ", ""),
                                          int(r.get("VGPR_Count") or 0),
                                          int(r.get("Accum_VGPR_Count") or 0),
                                          int(r.get("LDS_Block_Size") or 0),
                                          int(r.get("Scratch_Size") or 0),
                                          int(r.get("Workgroup_Size") or 0)))
        return vals, res
    ins, kres = per_family(insts_csv)
    busy, _ = per_family(busy_csv)
    fams = {}
    for k in ins:
        m = {c: sum(v) / len(v) for c, v in ins[k].items()}
        b = {c: sum(v) / len(v) for c, v in busy.get(k, {}).items()}
        f64 = m.get("SQ_INSTS_VALU_FMA_F64", 0) + m.get("SQ_INSTS_VALU_ADD_F64", 0) + \
            m.get("SQ_INSTS_VALU_MUL_F64", 0) + m.get("SQ_INSTS_VALU_TRANS_F64", 0)
        fams[k] = {"valu_insts_per_launch": m.get("SQ_INSTS_VALU"),
                   "fp64_insts_per_launch": f64,
                   "fp64_fma_per_launch": m.get("SQ_INSTS_VALU_FMA_F64"),
                   "fp64_trans_per_launch": m.get("SQ_INSTS_VALU_TRANS_F64"),
                   "fp64_flops_per_launch": 64 * (2 * m.get("SQ_INSTS_VALU_FMA_F64", 0) +
                                                  m.get("SQ_INSTS_VALU_ADD_F64", 0) +
                                                  m.get("SQ_INSTS_VALU_MUL_F64", 0)),
                   "fp64_share_of_valu": f64 / m["SQ_INSTS_VALU"] if m.get("SQ_INSTS_VALU") else None,
                   "waves_per_launch": m.get("SQ_WAVES"),
                   "valu_busy": b.get("VALUBusy", 0.0) / 100.0,
                   "valu_lane_utilization": b.get("VALUUtilization", 0.0) / 100.0,
                   "mean_occupancy_waves_per_simd": b.get("MeanOccupancyPerActiveCU"),
                   "kernels": [{"name": n, "vgpr": v, "agpr": a, "lds_bytes": lds,
                                "scratch_bytes": sc, "workgroup": wg}
                               for n, v, a, lds, sc, wg in sorted(kres[k])]}
    res = {"workload": workload, "source_sha256": source_hash(), "commands": commands,
           "families": fams}
    base = os.path.join(out_dir, "fp64_valu_%s" % workload)
    with open(base + ".json", "w") as f:
        json.dump(res, f, indent=1)
    lines = ["# FP64 VALU counters per launch, %s" % workload, "",
             "rocprofv3 --pmc runs (one per counter set):", ""] + \
        ["    " + c for c in commands] + [
        "", "Kernel sources sha256: `%s`" % res["source_sha256"], "",
        "VALU busy: share of the kernel's time the CUs' vector ALUs issue (VALUBusy); "
        "lane utilisation: active lanes per VALU instruction (VALUUtilization); FP64 FLOP "
        "= 64 x (2 FMA + ADD + MUL) wave instructions.", "",
        "| family | VALU insts | FP64 insts | FP64 share | FP64 GFLOP | VALU busy | lanes | "
        "waves/SIMD | VGPR (record) | LDS B | scratch B |", "|---|---|---|---|---|---|---|---|---|---|---|"]
    for k, v in sorted(fams.items()):
        ks = v["kernels"][0] if v["kernels"] else {}
        lines.append("| %s | %.3g | %.3g | %.2f | %.2f | %.2f | %.2f | %.1f | %s | %s | %s |" % (
            k, v["valu_insts_per_launch"] or 0, v["fp64_insts_per_launch"],
            v["fp64_share_of_valu"] or 0, v["fp64_flops_per_launch"] / 1e9, v["valu_busy"],
            v["valu_lane_utilization"], v["mean_occupancy_waves_per_simd"] or 0,
            ks.get("vgpr", "?"), ks.get("lds_bytes", "?"), ks.get("scratch_bytes", "?")))
    lines += ["", "waves/SIMD: MeanOccupancyPerActiveCU as rocprofv3 reports it (it reads 2.0 for "
              "a kernel the compiler limits to 2 waves per SIMD). VGPR (record): the dispatch "
              "record's VGPR_Count, which on gfx950 is half the compiler's per-lane count "
              "(the kernel-resource-usage remark).", "",
              "Kernels of each family (VGPRs, LDS and scratch per work-group from the "
              "dispatch records):", ""]
    for k, v in sorted(fams.items()):
        for ks in v["kernels"]:
            lines.append("- %s: `%s` VGPR %d, AGPR %d, LDS %d B, scratch %d B, work-group %d" % (
                k, ks["name"], ks["vgpr"], ks["agpr"], ks["lds_bytes"], ks["scratch_bytes"],
                ks["workgroup"]))
    with open(base + ".md", "w") as f:
        f.write("\n".join(lines) + "\n")
    return res


def kernel_family(name):
    """Kernel family of a device kernel name as rocprofv3 prints it."""
    if "k_ad_" in name or "k_curl" in name or "k_pack_sides" in name:
        for key, fam in (("k_ad_march_fused", "adj_march_fused"),
                         ("k_ad_row_fused", "adj_row_fused"),
                         ("k_ad_faces", "adj_faces"), ("k_ad_recon", "adj_recon"),
                         ("k_ad_prims", "adj_prims"), ("k_ad_edges", "adj_edges"),
                         ("k_pack_sides", "tape_sides"), ("k_curl", "curl")):
            if key in name:
                if fam == "adj_faces":
                    # k_ad_faces<D>: PCM stage; k_ad_faces_row / _march: reconstructing stage
                    return "adj_faces_recon" if ("_row" in name or "_march" in name) \
                        else "adj_faces_pcm"
                return fam
        return "adj_other"
    if "k_pred" in name:
        return "predictor"
    if "k_prims" in name:
        return "prims"
    if "k_ct_update" in name:
        return "ct_update"
    if "k_dt_" in name:
        return "dt"
    if "k_flux" in name:
        # template arguments <..., RECON>; RECON 1 is the PCM predictor
        targs = name[name.index("<") + 1:name.index(">")].replace(" ", "").split(",")
        return "flux_pcm_hlld" if targs[-1] == "1" else "flux_recon_hlld"
    if "copyBuffer" in name:
        return "copy"
    return None


def summarize_counters(fetch_csv, write_csv, copy_bytes, workload, commands, out_dir):
    """rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE (KiB per dispatch) -> calibrated
    HBM bytes per launch of each kernel family.  FETCH_SIZE and WRITE_SIZE are
    scaled by the factor that makes them read copy_bytes for the plain device
    copy the same runs made (the copy's dispatches are summed)."""
    import collections
    import csv

    def per_family(path):
        fam = collections.defaultdict(list)
        for r in csv.DictReader(open(path)):
            k = kernel_family(r["Kernel_Name"])
            if k:
                fam[k].append(float(r["Counter_Value"]) * 1024.0)
        return fam
    fe, wr = per_family(fetch_csv), per_family(write_csv)
    ffac = copy_bytes / sum(fe["copy"])
    wfac = copy_bytes / sum(wr["copy"])
    fams = {}
    for k in fe:
        if k == "copy":
            continue
        nf = len(fe[k])
        # dt is one launch of a partial and a final kernel
        per = 2 if k == "dt" else 1
        fb = ffac * sum(fe[k]) / (nf / per)
        wb = wfac * sum(wr[k]) / (len(wr[k]) / per)
        fams[k] = {"fetch_bytes_per_launch": fb, "write_bytes_per_launch": wb,
                   "traffic_bytes_per_launch": fb + wb, "dispatches": nf}
    res = {"workload": workload, "source_sha256": source_hash(),
           "calibration": {"copy_bytes": copy_bytes, "fetch_factor": ffac, "write_factor": wfac},
           "commands": commands, "families": fams}
    base = os.path.join(out_dir, "hbm_counters_%s" % workload)
    with open(base + ".json", "w") as f:
        json.dump(res, f, indent=1)
    lines = ["# HBM traffic per launch, %s" % workload, "",
             "rocprofv3 counters FETCH_SIZE and WRITE_SIZE (KiB per dispatch), each from its own run:",
             ""] + ["    " + c for c in commands] + [
             "", "Calibration: the same runs copy %d bytes device-to-device first; FETCH_SIZE reads "
             "%.3f of them (factor %.3f), WRITE_SIZE %.3f (factor %.3f)." % (
                 copy_bytes, 1 / ffac, ffac, 1 / wfac, wfac),
             "", "Kernel sources sha256: `%s`" % res["source_sha256"], "",
             "| kernel family | dispatches | read GiB/launch | write GiB/launch | total GB/launch |",
             "|---|---|---|---|---|"]
    for k, v in sorted(fams.items()):
        lines.append("| %s | %d | %.3f | %.3f | %.3f |" % (
            k, v["dispatches"], v["fetch_bytes_per_launch"] / 2**30,
            v["write_bytes_per_launch"] / 2**30, v["traffic_bytes_per_launch"] / 1e9))
    with open(base + ".md", "w") as f:
        f.write("\n".join(lines) + "\n")
    return res


def summarize_trace(stats_csv, workload, command, out_dir):
    """rocprofv3 --kernel-trace --stats kernel table -> markdown summary
    (profiles/kernel_trace_<workload>.md)."""
    import csv
    rows = list(csv.DictReader(open(stats_csv)))
    lines = ["# Kernel durations, %s" % workload, "", "    " + command, "",
             "Kernel sources sha256: `%s`" % source_hash(), "",
             "| kernel | family | calls | average ms | total ms | % |", "|---|---|---|---|---|---|"]
    for r in rows:
        fam = kernel_family(r["Name"])
        if fam in (None, "copy"):
            continue
        name = r["Name"].split("(")[0].replace("void ", "")
        lines.append("| `%s` | %s | %s | %.4f | %.3f | %s |" % (
            name, fam, r["Calls"], float(r["AverageNs"]) / 1e6,
            float(r["TotalDurationNs"]) / 1e6, r["Percentage"]))
    path = os.path.join(out_dir, "kernel_trace_%s.md" % workload)
    with open(path, "w") as f:
        f.write("\n".join(lines) + "\n")
    return path


def ensemble_bench(count, steps, warmup):
    """Config-4-style ensemble (`count` independent linear-wave runs of 16..96
    cells per axis): one vlct_step_batch per step against the same instances
    stepped one after another with vlct_step, both on the current stream with
    dt chained on the device; the two must agree bit for bit."""
    import numpy as np
    import torch
    from paper_2402_05240_amd import inputs as I
    from paper_2402_05240_amd.device import BatchStepper, Stepper
    ens = I.ensemble(count)
    grids = [g for g, _, _ in ens]
    states = [s for _, s, _ in ens]
    ncell = sum(g.ncells for g in grids)
    bs = BatchStepper(grids).upload(states)
    bs.compute_dt()
    singles = [Stepper(g).upload(s) for g, s in zip(grids, states)]
    for st in singles:
        st.compute_dt()

    def timed(fn, k):
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(k):
            fn()
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / k

    def seq_step():
        for st in singles:
            st.step()
    for _ in range(warmup):
        bs.step()
        seq_step()
    ms_batch = timed(bs.step, steps)
    ms_seq = timed(seq_step, steps)
    # the batched step captured into a HIP graph: two steps (A -> B -> A) per
    # replay, so host-side launch work leaves the timed loop
    gbs = BatchStepper(grids).upload(states)
    gbs.compute_dt()
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        gbs.step()
        gbs.step()
    graph.replay()
    ms_graph = timed(graph.replay, max(1, steps // 2)) / 2.0
    # per-instance tiles from the library's autotuner, timed like the default
    tuner = BatchStepper(grids).upload(states)
    tuner.compute_dt()
    plan = tuner.tune(reps=3)
    del tuner
    tbs = BatchStepper(grids, plan=plan).upload(states)
    tbs.compute_dt()
    for _ in range(warmup):
        tbs.step()
    ms_tuned = timed(tbs.step, steps)
    # config 4 proper: every instance to its own period, batched with
    # per-instance retirement (vlct_step_batch_until) against the instances
    # run one after another with the same clipped last step
    periods = [T for _, _, T in ens]
    ub = BatchStepper(grids, inplace=True).upload(states)
    ub.compute_dt()
    torch.cuda.synchronize()
    ea, eb = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ea.record()
    nbatch = ub.run_until(periods)
    eb.record()
    torch.cuda.synchronize()
    ms_until = ea.elapsed_time(eb)
    until_out = ub.download()
    del ub
    seq = [Stepper(g, inplace=True) for g in grids]

    def seq_run(counts=None):
        found = []
        for q, (st, s0, T) in enumerate(zip(seq, states, periods)):
            st.upload(s0)
            st.compute_dt()
            t = torch.zeros(1, dtype=torch.float64, device="cuda")
            te = torch.tensor([T], dtype=torch.float64, device="cuda")
            n = 0
            while (counts is None and float(t.item()) < T) or (counts is not None and n < counts[q]):
                dte = torch.minimum(st.dt, te - t)
                st.dt.copy_(dte)
                st.step()
                t += dte
                n += 1
            found.append(n)
        return found
    progress("ensemble: batched to one period each, %d batched steps" % nbatch)
    counts = seq_run()          # untimed: each instance's step count
    torch.cuda.synchronize()
    ea.record()
    seq_run(counts)             # timed: the same steps with no host round trip
    eb.record()
    torch.cuda.synchronize()
    ms_seq_until = ea.elapsed_time(eb)
    same_until = all(np.array_equal(o[f], st.download()[f]) for o, st in zip(until_out, seq)
                     for f in I.FIELDS)
    cell_steps = sum(g.ncells * n for g, n in zip(grids, counts))
    to_period = {"batched_until": {"ms": ms_until, "batched_steps": nbatch,
                                   "cell_updates_per_s": cell_steps / (ms_until * 1e-3)},
                 "sequential": {"ms": ms_seq_until,
                                "cell_updates_per_s": cell_steps / (ms_seq_until * 1e-3)},
                 "steps_per_instance": {"min": min(counts), "max": max(counts),
                                        "total": sum(counts)},
                 "speedup": ms_seq_until / ms_until, "bitwise_equal": bool(same_until)}
    del seq
    hist = {}
    for p in plan:
        key = "ct%dx%d_march%d" % ((64, 32, 16)[p & 15], (8, 16, 32)[p & 15], (16, 32, 8)[p >> 4])
        hist[key] = hist.get(key, 0) + 1
    outs = bs.download()
    same = all(np.array_equal(o[f], st.download()[f]) for o, st in zip(outs, singles)
               for f in I.FIELDS)
    same = same and all(np.array_equal(o[f], t[f]) for o, t in zip(outs, tbs.download())
                        for f in I.FIELDS)
    return {"workload": "ensemble_linear_%d" % count, "instances": count,
            "cells": ncell, "sizes": "16..96 per axis, non-cubic",
            "recon": "PLMC", "steps": steps, "warmup": warmup,
            "batched": {"ms_per_step": ms_batch, "cell_updates_per_s": ncell / (ms_batch * 1e-3)},
            "sequential": {"ms_per_step": ms_seq, "cell_updates_per_s": ncell / (ms_seq * 1e-3)},
            "batched_graph": {"ms_per_step": ms_graph,
                              "cell_updates_per_s": ncell / (ms_graph * 1e-3)},
            "batched_tuned": {"ms_per_step": ms_tuned,
                              "cell_updates_per_s": ncell / (ms_tuned * 1e-3), "plan": hist},
            "speedup": ms_seq / ms_batch, "speedup_tuned": ms_seq / ms_tuned,
            "bitwise_equal": bool(same), "to_one_period": to_period}


RECON_NAMES = {1: "PCM", 2: "PLMC", 3: "PPMC", 4: "PLMP", 5: "PPMP"}


def adjoint_bench(n, steps, warmup, recon=2):
    """Cost of the adjoint of one step against one forward step on decaying
    turbulence at n^3 (PLMC unless `recon` says otherwise): the forward step
    is vlct_step with the next-dt reduction, the adjoint is vlct_step_adjoint
    (which recomputes the forward intermediates it needs); both timed with
    events on the current stream."""
    import torch
    from paper_2402_05240_amd import inputs as I
    from paper_2402_05240_amd.device import Adjoint, Stepper
    g, s = I.turbulence((n, n, n), recon=recon)
    fwd = Stepper(g).upload(s)
    fwd.compute_dt()
    dt = float(fwd.dt.item())
    adj = Adjoint(g)
    adj.state.upload(s)
    for f in I.FIELDS:
        adj.lam_out.t[f].normal_()
    adj.dt.fill_(dt)

    def timed(fn, k):
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(k):
            fn()
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / k

    def fstep():
        fwd.set_dt(dt)
        fwd.step()
    # taped forward step and the adjoint from its tape
    from paper_2402_05240_amd import autograd as AG
    sim = AG.Simulator(g)
    fields = [adj.state.t[f] for f in I.FIELDS]
    lam = [adj.lam_out.t[f] for f in I.FIELDS]
    tape = sim.new_tape()

    def ftaped():
        sim.step_taped(fields, adj.dt, tape)

    def ataped():
        sim.adjoint_taped(fields, lam, adj.dt, tape)
    for _ in range(warmup):
        fstep()
        adj.run()
        ftaped()
        ataped()
    # interleaved rounds, the minimum of each
    rounds = {"forward": [], "adjoint": [], "taped_forward": [], "taped_adjoint": []}
    for _ in range(3):
        rounds["forward"].append(timed(fstep, steps))
        rounds["adjoint"].append(timed(adj.run, steps))
        rounds["taped_forward"].append(timed(ftaped, steps))
        rounds["taped_adjoint"].append(timed(ataped, steps))
    ms_f, ms_a = min(rounds["forward"]), min(rounds["adjoint"])
    ms_ft, ms_at = min(rounds["taped_forward"]), min(rounds["taped_adjoint"])
    name = RECON_NAMES[recon]
    return {"workload": "turbulence_%s_%d" % (name.lower(), n), "grid": [n, n, n], "recon": name,
            "steps": steps, "forward_ms": ms_f, "adjoint_ms": ms_a, "ratio": ms_a / ms_f,
            "taped_forward_ms": ms_ft, "taped_adjoint_ms": ms_at,
            "ratio_taped": ms_at / ms_f, "tape_bytes": sim.tape_bytes,
            "rounds_ms": rounds,
            "workspace_bytes": adj.ws_bytes,
            "note": "ratio: self-contained adjoint (recomputes the step's fluxes) / forward "
                    "step; ratio_taped: adjoint from the tape of a taped forward step "
                    "(vlct_step_taped, same kernels as the step plus the tape) / forward step"}


def inverse_bench(n, steps):
    """Differentiable turbulence inverse problem at n^3 (PLMC): parameters are
    the initial conserved variables and the edge vector potential A (B = b0 +
    curl_h A), the forward pass runs `steps` steps on the recorded CFL chain
    with sqrt(steps) checkpoints, loss = mean((rho_final - target)^2) for a
    seeded target field; the backward pass recomputes each segment and runs
    the step adjoints.  Times both passes with events on the current stream."""
    import numpy as np
    import torch
    from paper_2402_05240_amd import autograd as AG
    from paper_2402_05240_amd import inputs as I
    g, s, A, b0 = I.turbulence_potential((n, n, n))
    rng = np.random.default_rng(5240)
    x, y, z = I._centres(g)
    ph = rng.uniform(0.0, 2.0 * np.pi, 3)
    target = 1.0 + 0.05 * np.sin(2 * np.pi * x + ph[0]) * np.sin(2 * np.pi * y + ph[1]) \
        * np.sin(2 * np.pi * z + ph[2])
    sim = AG.Simulator(g)
    tgt = torch.from_numpy(target).cuda()

    def run(nsteps):
        cons = [torch.from_numpy(s[f]).cuda().requires_grad_(True)
                for f in ("rho", "mx", "my", "mz", "E")]
        pot = [torch.from_numpy(a).cuda().requires_grad_(True) for a in A]
        torch.cuda.synchronize()
        e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        e[0].record()
        bf = AG.curl(sim, *pot)
        out, _ = AG.rollout(sim, cons + [bf[0] + b0[0], bf[1], bf[2]], nsteps=nsteps)
        loss = ((out[0] - tgt) ** 2).mean()
        e[1].record()
        loss.backward()
        e[2].record()
        torch.cuda.synchronize()
        gn = math.sqrt(sum(float((q.grad ** 2).sum()) for q in cons + pot))
        return e[0].elapsed_time(e[1]), e[1].elapsed_time(e[2]), float(loss.item()), gn

    run(2)  # warm-up: workspaces and allocator
    torch.cuda.reset_peak_memory_stats()
    ms_f, ms_b, loss, gnorm = run(steps)
    seg = int(math.ceil(math.sqrt(steps)))
    return {"workload": "inverse_turbulence_plmc_%d" % n, "grid": [n, n, n], "steps": steps,
            "checkpoint_segment": seg, "forward_ms": ms_f, "backward_ms": ms_b,
            "ratio": ms_b / ms_f, "loss": loss, "grad_norm": gnorm,
            "peak_device_bytes": int(torch.cuda.max_memory_allocated()),
            "note": "backward = segment recomputation + one adjoint per step"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="turbulence_plmc_256", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-ensemble", action="store_true",
                    help="skip the batched-ensemble measurement (64 small runs)")
    ap.add_argument("--ensemble-steps", type=int, default=10)
    ap.add_argument("--no-adjoint", action="store_true",
                    help="skip the adjoint/forward cost measurement")
    ap.add_argument("--adjoint-n", type=int, nargs="*", default=[128],
                    help="cells per axis of the adjoint cost measurement(s)")
    ap.add_argument("--adjoint-steps", type=int, default=10)
    ap.add_argument("--no-inverse", action="store_true",
                    help="skip the differentiable inverse-problem measurement")
    ap.add_argument("--inverse-n", type=int, default=128)
    ap.add_argument("--inverse-steps", type=int, default=200)
    ap.add_argument("--adjoint-recon", default="plmc",
                    choices=["pcm", "plmc", "ppmc", "plmp", "ppmp"],
                    help="corrector reconstruction of the adjoint cost measurement")
    ap.add_argument("--no-workloads", action="store_true",
                    help="skip the other workloads (PPMC turbulence 256^3, blast 512^3, linear "
                         "wave 32^3)")
    ap.add_argument("--cpu-planes", type=int, default=256)
    ap.add_argument("--cpu-steps", type=int, default=3)
    ap.add_argument("--cpu-threads", type=int, default=0)
    ap.add_argument("--copy-calibration-gib", type=float, default=0.0,
                    help="first run one device-to-device copy of this many GiB (a plain copy "
                         "kernel of known size, to calibrate HBM byte counters)")
    ap.add_argument("--summarize-counters", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="write profiles/hbm_counters_<workload>.{json,md} from the two "
                         "rocprofv3 --pmc runs (no GPU needed)")
    ap.add_argument("--summarize-valu", nargs=2, metavar=("INSTS_CSV", "BUSY_CSV"),
                    help="write profiles/fp64_valu_<workload>.{json,md} from the two rocprofv3 "
                         "--pmc runs of FP64 VALU counters (no GPU needed)")
    ap.add_argument("--summarize-trace", metavar="KERNEL_STATS_CSV",
                    help="write profiles/kernel_trace_<workload>.md (no GPU needed)")
    ap.add_argument("--trace-name", default=None,
                    help="name of the --summarize-trace output (default: the workload)")
    ap.add_argument("--commands", nargs="*", default=[],
                    help="the rocprofv3 command lines the summarised files came from")
    args = ap.parse_args()
    if args.summarize_counters or args.summarize_trace or args.summarize_valu:
        out_dir = os.path.join(ROOT, "profiles")
        os.makedirs(out_dir, exist_ok=True)
        if args.summarize_counters:
            summarize_counters(args.summarize_counters[0], args.summarize_counters[1],
                               int(args.copy_calibration_gib * (1 << 30)) or (1 << 30),
                               args.workload, args.commands[:2], out_dir)
        if args.summarize_valu:
            summarize_valu(args.summarize_valu[0], args.summarize_valu[1], args.workload,
                           args.commands[:2], out_dir)
        if args.summarize_trace:
            summarize_trace(args.summarize_trace, args.trace_name or args.workload,
                            args.commands[-1] if args.commands else "", out_dir)
        return
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
    e0, e1 = events.new(), events.new()
    torch.cuda.synchronize()
    # the headline: plain vlct_step calls, nothing else in the timed loop
    w0 = time.perf_counter()
    events.record(e0, stream.cuda_stream)
    for _ in range(args.steps):
        st.step()
    events.record(e1, stream.cuda_stream)
    torch.cuda.synchronize()
    w1 = time.perf_counter()
    ms_total = events.elapsed_ms(e0, e1)
    status = st.status_bits()
    # per-kernel times from a second pass of as many steps through
    # vlct_step_observed, each kernel family bracketed with HIP events on the
    # stream the library launches it on
    timer = KernelTimer(vlct, events)
    timer.active = True
    for _ in range(args.steps):
        st.step_observed(timer)
    torch.cuda.synchronize()
    timer.active = False
    kern = timer.summary()

    ncell = g.ncells
    ms_step = ms_total / args.steps
    value = ncell * args.steps / (ms_total * 1e-3)
    rl = rooflines(g, kern, args.steps, args.workload)
    dom = max(rl, key=lambda k: rl[k]["ms_per_step"])
    recon_name = RECON_NAMES[g.recon]
    design_bytes = sum(r["bytes_per_step"] for r in rl.values() if "bytes_per_step" in r) / ncell
    out = {
        "metric": HEADLINE_METRIC,
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
        # the dominant kernel family (most time per step) against the roof
        # its counters say binds it
        "roofline": rl[dom],
        "rooflines": rl,
        # the whole step against the HBM roofline: the scope's algorithmic
        # bytes (state in and out once, 128 B per cell update), the bytes this
        # design's kernels are written to move, and what the HBM counters saw
        "step_roofline": step_roofline(rl, value, ncell, design_bytes),
        "adjoint_forward_cost": None,
        "kernels_ms_per_step": {k: v["total_ms"] / args.steps for k, v in kern.items()},
        "wall_ms_per_step": (w1 - w0) * 1e3 / args.steps,
        "status": status,
    }
    del st
    torch.cuda.empty_cache()
    progress("headline %s: %.3f ms per step" % (args.workload, ms_step))
    if not args.no_adjoint:
        recon = {v.lower(): k for k, v in RECON_NAMES.items()}[args.adjoint_recon]
        costs = [adjoint_bench(n, args.adjoint_steps, 2, recon) for n in args.adjoint_n]
        out["adjoint_forward_cost"] = costs[0] if len(costs) == 1 else costs
        torch.cuda.empty_cache()
        progress("adjoint cost")
    if not args.no_inverse:
        out["inverse_problem"] = inverse_bench(args.inverse_n, args.inverse_steps)
        torch.cuda.empty_cache()
        progress("inverse problem")
    if not args.no_ensemble:
        torch.cuda.empty_cache()
        out["ensemble"] = ensemble_bench(64, args.ensemble_steps, 2)
        progress("ensemble")
    if not args.no_workloads:
        torch.cuda.empty_cache()
        out["workloads"] = {}
        for name in ("turbulence_ppmc_256", "blast_ppmc_512", "linear_fast_32"):
            if name != args.workload:
                out["workloads"][name] = workload_bench(name)
                torch.cuda.empty_cache()
                progress("workload %s" % name)
    if not args.no_cpu_baseline:
        torch.cuda.empty_cache()
        threads = args.cpu_threads or min(16, os.cpu_count() or 1)
        out["cpu_baseline"] = cpu_baseline(g, s0, args.cpu_planes, args.cpu_steps, threads)
        # the same oracle on one host thread, on a thinner slab of the same state
        one = cpu_baseline(g, s0, max(1, args.cpu_planes // 16), args.cpu_steps, 1)
        out["cpu_baseline"]["one_thread"] = one
        progress("cpu baseline")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
