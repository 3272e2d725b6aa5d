"""ctypes wrapper of the CPU oracle (oracle/libvlct_ref.so).

TEST INFRASTRUCTURE ONLY: the oracle checks the GPU library and must never be
used by it.  Only the tests, the smoke entry point and the benchmark's
CPU-baseline leg may import this module.
"""
from __future__ import annotations

import ctypes
import os
from typing import Dict, Tuple

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libvlct_ref.so")
FIELDS = ("rho", "mx", "my", "mz", "E", "bx", "by", "bz")

STATUS_PRESSURE_FLOOR = 1
STATUS_DENSITY_FLOOR = 2
STATUS_NONFINITE = 4


class _Grid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("dx", ctypes.c_double), ("dy", ctypes.c_double), ("dz", ctypes.c_double),
                ("gamma", ctypes.c_double), ("cfl", ctypes.c_double),
                ("recon", ctypes.c_int32), ("bc", ctypes.c_int32 * 3)]


_DP = ctypes.POINTER(ctypes.c_double)
_lib = None


def load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build as _b  # noqa: F401  (package-relative when imported as oracle)
        _lib = ctypes.CDLL(LIB_PATH)
        _lib.vref_step.argtypes = [ctypes.POINTER(_Grid), ctypes.POINTER(_DP), ctypes.POINTER(_DP),
                                   ctypes.c_double, _DP, ctypes.POINTER(ctypes.c_uint32),
                                   ctypes.c_int]
        _lib.vref_step.restype = ctypes.c_int
        _lib.vref_cfl_dt.argtypes = [ctypes.POINTER(_Grid), ctypes.POINTER(_DP), _DP, ctypes.c_int]
        _lib.vref_cfl_dt.restype = ctypes.c_int
        _lib.vref_wave_speeds.argtypes = [ctypes.c_double] * 6 + [_DP, _DP]
        _lib.vref_hlld.argtypes = [_DP, _DP, ctypes.c_double, ctypes.c_double, _DP]
        _lib.vref_phys_flux.argtypes = [_DP, ctypes.c_double, ctypes.c_double, _DP]
        _lib.vref_eigen.argtypes = [_DP, ctypes.c_double, ctypes.c_double, _DP, _DP, _DP]
        _lib.vref_plmc.argtypes = [_DP, ctypes.c_double, ctypes.c_double, _DP, _DP]
        _lib.vref_ppmc.argtypes = [_DP, ctypes.c_double, ctypes.c_double, _DP, _DP]
        _lib.vref_plmp.argtypes = [_DP, _DP, _DP]
        _lib.vref_ppmp.argtypes = [_DP, ctypes.c_double, ctypes.c_double, _DP, _DP]
        _lib.vref_ct_update.argtypes = [ctypes.POINTER(_Grid), ctypes.POINTER(_DP),
                                        ctypes.POINTER(_DP), _DP, _DP, _DP, ctypes.c_double]
        _lib.vref_edge_emfs.argtypes = [ctypes.POINTER(_Grid), ctypes.POINTER(_DP), ctypes.c_int,
                                        _DP, _DP, _DP, ctypes.c_int]
        _lib.vref_edge_emfs.restype = ctypes.c_int
        _lib.vref_stage_fluxes.argtypes = [ctypes.POINTER(_Grid), ctypes.POINTER(_DP), ctypes.c_int,
                                           ctypes.POINTER(_DP), ctypes.POINTER(_DP),
                                           ctypes.POINTER(_DP), ctypes.c_int]
        _lib.vref_stage_fluxes.restype = ctypes.c_int
        _lib.vref_half_step.argtypes = [ctypes.POINTER(_Grid), ctypes.POINTER(_DP),
                                        ctypes.POINTER(_DP), ctypes.c_double, ctypes.c_int]
        _lib.vref_half_step.restype = ctypes.c_int
        _lib.vref_divb_norm.argtypes = [ctypes.POINTER(_Grid), ctypes.POINTER(_DP)]
        _lib.vref_divb_norm.restype = ctypes.c_double
    return _lib


def _grid(g) -> _Grid:
    cg = _Grid()
    cg.nx, cg.ny, cg.nz = int(g.nx), int(g.ny), int(g.nz)
    cg.dx, cg.dy, cg.dz = float(g.dx), float(g.dy), float(g.dz)
    cg.gamma, cg.cfl = float(g.gamma), float(g.cfl)
    cg.recon = int(g.recon)
    for d in range(3):
        cg.bc[d] = int(g.bc[d])
    return cg


def _ptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(_DP)


def _vec(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _check_state(g, s: Dict[str, np.ndarray]):
    for f in FIELDS:
        if s[f].shape != g.field_shape(f):
            raise ValueError("field %s has shape %s, expected %s" % (f, s[f].shape, g.field_shape(f)))


def step(g, s: Dict[str, np.ndarray], dt: float, nthreads: int = 0,
         inplace: bool = False) -> Tuple[Dict[str, np.ndarray], float, int]:
    """One VL+CT step; returns (new_state, next_dt, status)."""
    lib = load()
    _check_state(g, s)
    src = {f: np.ascontiguousarray(s[f], dtype=np.float64) for f in FIELDS}
    dst = src if inplace else {f: np.empty_like(src[f]) for f in FIELDS}
    inp = (_DP * 8)(*[_ptr(src[f]) for f in FIELDS])
    out = (_DP * 8)(*[_ptr(dst[f]) for f in FIELDS])
    nd = ctypes.c_double(0.0)
    st = ctypes.c_uint32(0)
    cg = _grid(g)
    rc = lib.vref_step(ctypes.byref(cg), inp, out, float(dt), ctypes.byref(nd), ctypes.byref(st),
                       int(nthreads))
    if rc != 0:
        raise ValueError("vref_step failed with code %d" % rc)
    return dst, nd.value, st.value


def cfl_dt(g, s: Dict[str, np.ndarray], nthreads: int = 0) -> float:
    lib = load()
    _check_state(g, s)
    src = {f: np.ascontiguousarray(s[f], dtype=np.float64) for f in FIELDS}
    inp = (_DP * 8)(*[_ptr(src[f]) for f in FIELDS])
    dt = ctypes.c_double(0.0)
    cg = _grid(g)
    rc = lib.vref_cfl_dt(ctypes.byref(cg), inp, ctypes.byref(dt), int(nthreads))
    if rc != 0:
        raise ValueError("vref_cfl_dt failed with code %d" % rc)
    return dt.value


def run(g, s, nsteps: int, dt0: float = None, nthreads: int = 0, t_end: float = None):
    """Advance nsteps (or to t_end, clipping the last dt); returns
    (state, dts, status) with the dt sequence actually used."""
    dt = cfl_dt(g, s, nthreads) if dt0 is None else dt0
    dts = []
    status = 0
    t = 0.0
    k = 0
    while True:
        if t_end is not None:
            if t >= t_end * (1 - 1e-14):
                break
            if t + dt > t_end:
                dt = t_end - t
        elif k >= nsteps:
            break
        s, nd, st = step(g, s, dt, nthreads)
        status |= st
        dts.append(dt)
        t += dt
        dt = nd
        k += 1
    return s, dts, status


def wave_speeds(rho, p, bn, bt1, bt2, gamma):
    lib = load()
    cf = ctypes.c_double()
    cs = ctypes.c_double()
    lib.vref_wave_speeds(rho, p, bn, bt1, bt2, gamma, ctypes.byref(cf), ctypes.byref(cs))
    return cf.value, cs.value


def hlld(wl, wr, bn, gamma, with_upwind: bool = False) -> np.ndarray:
    """HLLD flux (7 components); with_upwind adds the CT upwind indicator."""
    lib = load()
    wl, wr = _vec(wl), _vec(wr)
    f = np.zeros(8)
    lib.vref_hlld(_ptr(wl), _ptr(wr), float(bn), float(gamma), _ptr(f))
    return f if with_upwind else f[:7].copy()


def phys_flux(w, bn, gamma) -> np.ndarray:
    lib = load()
    w = _vec(w)
    f = np.zeros(7)
    lib.vref_phys_flux(_ptr(w), float(bn), float(gamma), _ptr(f))
    return f


def eigen(w, bn, gamma):
    lib = load()
    w = _vec(w)
    R = np.zeros(49)
    L = np.zeros(49)
    lam = np.zeros(7)
    lib.vref_eigen(_ptr(w), float(bn), float(gamma), _ptr(R), _ptr(L), _ptr(lam))
    return R.reshape(7, 7), L.reshape(7, 7), lam


def plmc(stencil, bn, gamma):
    """stencil: (3, 7) primitives of cells i-1, i, i+1 -> (face_minus, face_plus)."""
    lib = load()
    st = _vec(stencil).reshape(-1)
    assert st.size == 21
    fm = np.zeros(7)
    fp = np.zeros(7)
    lib.vref_plmc(_ptr(st), float(bn), float(gamma), _ptr(fm), _ptr(fp))
    return fm, fp


def ppmc(stencil, bn, gamma):
    """stencil: (5, 7) primitives of cells i-2..i+2 -> (face_minus, face_plus)."""
    lib = load()
    st = _vec(stencil).reshape(-1)
    assert st.size == 35
    fm = np.zeros(7)
    fp = np.zeros(7)
    lib.vref_ppmc(_ptr(st), float(bn), float(gamma), _ptr(fm), _ptr(fp))
    return fm, fp


def plmp(stencil):
    """Primitive-limited PLM: stencil (3, 7) -> (face_minus, face_plus)."""
    lib = load()
    st = _vec(stencil).reshape(-1)
    assert st.size == 21
    fm = np.zeros(7)
    fp = np.zeros(7)
    lib.vref_plmp(_ptr(st), _ptr(fm), _ptr(fp))
    return fm, fp


def ppmp(stencil, bn, gamma):
    """Primitive-limited PPM: stencil (5, 7) -> (face_minus, face_plus)."""
    lib = load()
    st = _vec(stencil).reshape(-1)
    assert st.size == 35
    fm = np.zeros(7)
    fp = np.zeros(7)
    lib.vref_ppmp(_ptr(st), float(bn), float(gamma), _ptr(fm), _ptr(fp))
    return fm, fp


def edge_shapes(g):
    nx, ny, nz = g.nx, g.ny, g.nz
    return {"ex": (nz + 1, ny + 1, nx), "ey": (nz + 1, ny, nx + 1), "ez": (nz, ny + 1, nx + 1)}


def ct_update(g, b: Tuple[np.ndarray, np.ndarray, np.ndarray], ex, ey, ez, dt):
    lib = load()
    bin_ = [np.ascontiguousarray(x, dtype=np.float64) for x in b]
    bout = [np.empty_like(x) for x in bin_]
    ex, ey, ez = _vec(ex), _vec(ey), _vec(ez)
    cg = _grid(g)
    lib.vref_ct_update(ctypes.byref(cg), (_DP * 3)(*[_ptr(x) for x in bin_]),
                       (_DP * 3)(*[_ptr(x) for x in bout]), _ptr(ex), _ptr(ey), _ptr(ez),
                       float(dt))
    return tuple(bout)


def edge_emfs(g, s, recon: int, nthreads: int = 0):
    lib = load()
    _check_state(g, s)
    src = {f: np.ascontiguousarray(s[f], dtype=np.float64) for f in FIELDS}
    inp = (_DP * 8)(*[_ptr(src[f]) for f in FIELDS])
    sh = edge_shapes(g)
    e = {k: np.zeros(v) for k, v in sh.items()}
    cg = _grid(g)
    rc = lib.vref_edge_emfs(ctypes.byref(cg), inp, int(recon), _ptr(e["ex"]), _ptr(e["ey"]),
                            _ptr(e["ez"]), int(nthreads))
    if rc != 0:
        raise ValueError("vref_edge_emfs failed")
    return e["ex"], e["ey"], e["ez"]


def divb_norm(g, s) -> float:
    lib = load()
    src = {f: np.ascontiguousarray(s[f], dtype=np.float64) for f in FIELDS}
    inp = (_DP * 8)(*[_ptr(src[f]) for f in FIELDS])
    cg = _grid(g)
    return lib.vref_divb_norm(ctypes.byref(cg), inp)


def half_step(g, s, dt, nthreads: int = 0):
    """Predictor only: the half-step state of a step of size dt."""
    lib = load()
    _check_state(g, s)
    src = {f: np.ascontiguousarray(s[f], dtype=np.float64) for f in FIELDS}
    dst = {f: np.empty_like(src[f]) for f in FIELDS}
    cg = _grid(g)
    rc = lib.vref_half_step(ctypes.byref(cg), (_DP * 8)(*[_ptr(src[f]) for f in FIELDS]),
                            (_DP * 8)(*[_ptr(dst[f]) for f in FIELDS]), float(dt), int(nthreads))
    if rc != 0:
        raise ValueError("vref_half_step failed")
    return dst


def stage_fluxes(g, s, recon: int, nthreads: int = 0):
    """Face fluxes of one stage: {axis: (8, *face_shape)} with the 7 sweep-frame
    components and the CT upwind indicator."""
    lib = load()
    _check_state(g, s)
    src = {f: np.ascontiguousarray(s[f], dtype=np.float64) for f in FIELDS}
    out = {d: np.zeros((8,) + g.field_shape(("bx", "by", "bz")[d])) for d in range(3)}
    arrs = {d: (_DP * 8)(*[_ptr(out[d][c]) for c in range(8)]) for d in range(3)}
    cg = _grid(g)
    rc = lib.vref_stage_fluxes(ctypes.byref(cg), (_DP * 8)(*[_ptr(src[f]) for f in FIELDS]),
                               int(recon), arrs[0], arrs[1], arrs[2], int(nthreads))
    if rc != 0:
        raise ValueError("vref_stage_fluxes failed")
    return out
