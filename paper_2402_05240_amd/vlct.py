"""Python binding of the C ABI in include/vlct.h (argument marshalling only).

Every step of the VL+CT integrator runs in the gfx950 library libvlct.so;
PyTorch supplies device memory and the stream.  The binding refuses to run if
the library is missing: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libvlct.so")

VLCT_OK = 0
VLCT_EINVAL = 1
VLCT_EWORKSPACE = 2
VLCT_EHIP = 3
VLCT_EUNSUPPORTED = 4
VLCT_ESCRATCH = 5
VLCT_NOALLOC_SCRATCH_BYTES = 64 << 20
VLCT_RECON_PCM = 1
VLCT_RECON_PLMC = 2
VLCT_RECON_PPMC = 3
VLCT_RECON_PLMP = 4
VLCT_RECON_PPMP = 5
VLCT_BC_PERIODIC = 0
VLCT_BC_OUTFLOW = 1
VLCT_STATUS_PRESSURE_FLOOR = 1
VLCT_STATUS_DENSITY_FLOOR = 2
VLCT_STATUS_NONFINITE = 4

EXPORTED = ("vlct_workspace_bytes", "vlct_cfl_dt", "vlct_step", "vlct_strerror",
            "vlct_abi_version", "vlct_step_observed", "vlct_kernel_name",
            "vlct_batch_workspace_bytes", "vlct_step_batch", "vlct_adjoint_workspace_bytes",
            "vlct_step_adjoint", "vlct_curl_potential", "vlct_curl_potential_adjoint",
            "vlct_tape_bytes", "vlct_step_taped", "vlct_adjoint_taped_workspace_bytes",
            "vlct_step_adjoint_taped", "vlct_step_batch_plan", "vlct_batch_tune",
            "vlct_step_noalloc", "vlct_step_batch_until")

VLCT_KERNEL_PRIMS = 0
VLCT_KERNEL_FLUX_PCM = 1
VLCT_KERNEL_FLUX_RECON = 2
VLCT_KERNEL_EDGES = 3
VLCT_KERNEL_UPDATE_HALF = 4
VLCT_KERNEL_UPDATE_FULL = 5
VLCT_KERNEL_DT = 6
VLCT_KERNEL_DT_FINAL = 7
VLCT_KERNEL_PREDICTOR = 8
VLCT_KERNEL_COUNT = 9

vlct_launch_observer = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_int, ctypes.c_int,
                                        ctypes.c_void_p)


class vlct_grid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("dx", ctypes.c_double), ("dy", ctypes.c_double), ("dz", ctypes.c_double),
                ("gamma", ctypes.c_double), ("cfl", ctypes.c_double),
                ("recon", ctypes.c_int32), ("bc", ctypes.c_int32 * 3)]


class vlct_state(ctypes.Structure):
    _fields_ = [(name, ctypes.c_void_p) for name in ("rho", "mx", "my", "mz", "E", "bx", "by", "bz")]


class VlctError(RuntimeError):
    def __init__(self, code: int, where: str):
        super().__init__("%s failed: %s (code %d)" % (where, vlct_strerror(code), code))
        self.code = code


_lib = None


def load(path: str = LIB_PATH):
    """Load libvlct.so; raises if it has not been built.

    torch is imported first when it is installed: it ships its own HIP
    runtime under the same soname, and the library must bind to that one
    copy, or the streams and device memory torch hands over would belong to a
    second runtime in the same process."""
    global _lib
    if _lib is None:
        if not os.path.exists(path):
            raise RuntimeError("libvlct.so not found at %s: build it with "
                               "`python -m paper_2402_05240_amd.build`" % path)
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        lib = ctypes.CDLL(path)
        lib.vlct_workspace_bytes.argtypes = [ctypes.POINTER(vlct_grid)]
        lib.vlct_workspace_bytes.restype = ctypes.c_size_t
        lib.vlct_cfl_dt.argtypes = [ctypes.POINTER(vlct_grid), ctypes.POINTER(vlct_state),
                                    ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                                    ctypes.c_void_p]
        lib.vlct_cfl_dt.restype = ctypes.c_int
        lib.vlct_step.argtypes = [ctypes.POINTER(vlct_grid), ctypes.POINTER(vlct_state),
                                  ctypes.POINTER(vlct_state), ctypes.c_void_p, ctypes.c_void_p,
                                  ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                                  ctypes.c_void_p]
        lib.vlct_step.restype = ctypes.c_int
        lib.vlct_step_noalloc.argtypes = [ctypes.POINTER(vlct_grid), ctypes.POINTER(vlct_state),
                                          ctypes.POINTER(vlct_state), ctypes.c_void_p,
                                          ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
        lib.vlct_step_noalloc.restype = ctypes.c_int
        lib.vlct_batch_workspace_bytes.argtypes = [ctypes.POINTER(vlct_grid), ctypes.c_int]
        lib.vlct_batch_workspace_bytes.restype = ctypes.c_size_t
        lib.vlct_step_batch.argtypes = [ctypes.c_int, ctypes.POINTER(vlct_grid),
                                        ctypes.POINTER(vlct_state), ctypes.POINTER(vlct_state),
                                        ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                        ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]
        lib.vlct_step_batch.restype = ctypes.c_int
        lib.vlct_step_batch_plan.argtypes = [ctypes.c_int, ctypes.POINTER(vlct_grid),
                                             ctypes.POINTER(vlct_state), ctypes.POINTER(vlct_state),
                                             ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                             ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                                             ctypes.c_void_p]
        lib.vlct_step_batch_plan.restype = ctypes.c_int
        lib.vlct_step_batch_until.argtypes = [ctypes.c_int, ctypes.POINTER(vlct_grid),
                                              ctypes.POINTER(vlct_state), ctypes.c_void_p,
                                              ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                              ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                              ctypes.c_size_t, ctypes.c_void_p]
        lib.vlct_step_batch_until.restype = ctypes.c_int
        lib.vlct_batch_tune.argtypes = [ctypes.c_int, ctypes.POINTER(vlct_grid),
                                        ctypes.POINTER(vlct_state), ctypes.POINTER(vlct_state),
                                        ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                                        ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p]
        lib.vlct_batch_tune.restype = ctypes.c_int
        lib.vlct_adjoint_workspace_bytes.argtypes = [ctypes.POINTER(vlct_grid)]
        lib.vlct_adjoint_workspace_bytes.restype = ctypes.c_size_t
        lib.vlct_step_adjoint.argtypes = [ctypes.POINTER(vlct_grid), ctypes.POINTER(vlct_state),
                                          ctypes.POINTER(vlct_state), ctypes.POINTER(vlct_state),
                                          ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                                          ctypes.c_void_p]
        lib.vlct_step_adjoint.restype = ctypes.c_int
        for name in ("vlct_tape_bytes", "vlct_adjoint_taped_workspace_bytes"):
            fn = getattr(lib, name)
            fn.argtypes = [ctypes.POINTER(vlct_grid)]
            fn.restype = ctypes.c_size_t
        lib.vlct_step_taped.argtypes = [ctypes.POINTER(vlct_grid), ctypes.POINTER(vlct_state),
                                        ctypes.POINTER(vlct_state), ctypes.c_void_p, ctypes.c_void_p,
                                        ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                                        ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]
        lib.vlct_step_taped.restype = ctypes.c_int
        lib.vlct_step_adjoint_taped.argtypes = [ctypes.POINTER(vlct_grid)] + \
            [ctypes.POINTER(vlct_state)] * 3 + [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                                                ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]
        lib.vlct_step_adjoint_taped.restype = ctypes.c_int
        for name in ("vlct_curl_potential", "vlct_curl_potential_adjoint"):
            fn = getattr(lib, name)
            fn.argtypes = [ctypes.POINTER(vlct_grid)] + [ctypes.c_void_p] * 7
            fn.restype = ctypes.c_int
        lib.vlct_strerror.argtypes = [ctypes.c_int]
        lib.vlct_strerror.restype = ctypes.c_char_p
        lib.vlct_abi_version.argtypes = []
        lib.vlct_abi_version.restype = ctypes.c_int
        lib.vlct_step_observed.argtypes = [ctypes.POINTER(vlct_grid), ctypes.POINTER(vlct_state),
                                           ctypes.POINTER(vlct_state), ctypes.c_void_p,
                                           ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                           ctypes.c_size_t, ctypes.c_void_p, vlct_launch_observer,
                                           ctypes.c_void_p]
        lib.vlct_step_observed.restype = ctypes.c_int
        lib.vlct_kernel_name.argtypes = [ctypes.c_int]
        lib.vlct_kernel_name.restype = ctypes.c_char_p
        _lib = lib
    return _lib


def make_grid(g) -> vlct_grid:
    """vlct_grid from any object with nx, ny, nz, dx, dy, dz, gamma, cfl, recon, bc."""
    cg = vlct_grid()
    cg.nx, cg.ny, cg.nz = int(g.nx), int(g.ny), int(g.nz)
    cg.dx, cg.dy, cg.dz = float(g.dx), float(g.dy), float(g.dz)
    cg.gamma, cg.cfl, cg.recon = float(g.gamma), float(g.cfl), int(g.recon)
    for d in range(3):
        cg.bc[d] = int(g.bc[d])
    return cg


def make_state(ptrs) -> vlct_state:
    """vlct_state from 8 device addresses (rho, mx, my, mz, E, bx, by, bz)."""
    st = vlct_state()
    for name, p in zip(("rho", "mx", "my", "mz", "E", "bx", "by", "bz"), ptrs):
        setattr(st, name, int(p) if p else None)
    return st


def vlct_workspace_bytes(grid: vlct_grid) -> int:
    return int(load().vlct_workspace_bytes(ctypes.byref(grid)))


def vlct_cfl_dt(grid: vlct_grid, state: vlct_state, dt_dev: int, ws: int, ws_bytes: int,
                stream: int) -> int:
    return int(load().vlct_cfl_dt(ctypes.byref(grid), ctypes.byref(state), dt_dev, ws,
                                  ws_bytes, stream))


def vlct_step(grid: vlct_grid, state_in: vlct_state, state_out: vlct_state, dt_dev: int,
              next_dt_dev: int, status_dev: int, ws: int, ws_bytes: int, stream: int) -> int:
    return int(load().vlct_step(ctypes.byref(grid), ctypes.byref(state_in),
                                ctypes.byref(state_out), dt_dev, next_dt_dev, status_dev, ws,
                                ws_bytes, stream))


def vlct_step_noalloc(grid: vlct_grid, state_in: vlct_state, state_out: vlct_state, dt_dev: int,
                      next_dt_dev: int, status_dev: int, stream: int) -> int:
    return int(load().vlct_step_noalloc(ctypes.byref(grid), ctypes.byref(state_in),
                                        ctypes.byref(state_out), dt_dev, next_dt_dev, status_dev,
                                        stream))


def vlct_batch_workspace_bytes(grids) -> int:
    """grids: sequence of vlct_grid."""
    arr = (vlct_grid * len(grids))(*grids)
    return int(load().vlct_batch_workspace_bytes(arr, len(grids)))


def vlct_step_batch(grids, states_in, states_out, dt_dev: int, next_dt_dev: int,
                    status_dev: int, ws: int, ws_bytes: int, stream: int) -> int:
    """grids, states_in, states_out: sequences of vlct_grid / vlct_state (host
    descriptors); dt_dev, next_dt_dev, status_dev: device arrays of len(grids)."""
    n = len(grids)
    g = (vlct_grid * n)(*grids)
    a = (vlct_state * n)(*states_in)
    b = (vlct_state * n)(*states_out)
    return int(load().vlct_step_batch(n, g, a, b, dt_dev, next_dt_dev, status_dev, ws, ws_bytes,
                                      stream))


def vlct_adjoint_workspace_bytes(grid: vlct_grid) -> int:
    return int(load().vlct_adjoint_workspace_bytes(ctypes.byref(grid)))


def vlct_step_adjoint(grid: vlct_grid, state_in: vlct_state, lam_out: vlct_state,
                      lam_in: vlct_state, dt_dev: int, ws: int, ws_bytes: int,
                      stream: int) -> int:
    return int(load().vlct_step_adjoint(ctypes.byref(grid), ctypes.byref(state_in),
                                        ctypes.byref(lam_out), ctypes.byref(lam_in), dt_dev, ws,
                                        ws_bytes, stream))


def vlct_tape_bytes(grid: vlct_grid) -> int:
    return int(load().vlct_tape_bytes(ctypes.byref(grid)))


def vlct_adjoint_taped_workspace_bytes(grid: vlct_grid) -> int:
    return int(load().vlct_adjoint_taped_workspace_bytes(ctypes.byref(grid)))


def vlct_step_taped(grid: vlct_grid, state_in: vlct_state, state_out: vlct_state, dt_dev: int,
                    next_dt_dev: int, status_dev: int, ws: int, ws_bytes: int, tape: int,
                    tape_bytes: int, stream: int) -> int:
    return int(load().vlct_step_taped(ctypes.byref(grid), ctypes.byref(state_in),
                                      ctypes.byref(state_out), dt_dev, next_dt_dev, status_dev,
                                      ws, ws_bytes, tape, tape_bytes, stream))


def vlct_step_adjoint_taped(grid: vlct_grid, state_in: vlct_state, lam_out: vlct_state,
                            lam_in: vlct_state, dt_dev: int, tape: int, tape_bytes: int, ws: int,
                            ws_bytes: int, stream: int) -> int:
    return int(load().vlct_step_adjoint_taped(ctypes.byref(grid), ctypes.byref(state_in),
                                              ctypes.byref(lam_out), ctypes.byref(lam_in), dt_dev,
                                              tape, tape_bytes, ws, ws_bytes, stream))


def vlct_curl_potential(grid: vlct_grid, ax: int, ay: int, az: int, bx: int, by: int, bz: int,
                        stream: int) -> int:
    return int(load().vlct_curl_potential(ctypes.byref(grid), ax, ay, az, bx, by, bz, stream))


def vlct_curl_potential_adjoint(grid: vlct_grid, lbx: int, lby: int, lbz: int, lax: int,
                                lay: int, laz: int, stream: int) -> int:
    return int(load().vlct_curl_potential_adjoint(ctypes.byref(grid), lbx, lby, lbz, lax, lay,
                                                  laz, stream))


def vlct_step_batch_plan(grids, states_in, states_out, dt_dev: int, next_dt_dev: int,
                         status_dev: int, plan, ws: int, ws_bytes: int, stream: int) -> int:
    """vlct_step_batch with a per-instance tile plan (sequence of ints or None)."""
    n = len(grids)
    g = (vlct_grid * n)(*grids)
    a = (vlct_state * n)(*states_in)
    b = (vlct_state * n)(*states_out)
    p = (ctypes.c_uint8 * n)(*plan) if plan is not None else None
    return int(load().vlct_step_batch_plan(n, g, a, b, dt_dev, next_dt_dev, status_dev,
                                           ctypes.cast(p, ctypes.c_void_p) if p is not None else None,
                                           ws, ws_bytes, stream))


def vlct_step_batch_until(grids, states, dt_dev: int, next_dt_dev: int, status_dev: int,
                          t_dev: int, t_end_dev: int, plan, ws: int, ws_bytes: int,
                          stream: int) -> int:
    """In-place batched step of the instances with t < t_end (device arrays)."""
    n = len(grids)
    g = (vlct_grid * n)(*grids)
    a = (vlct_state * n)(*states)
    p = (ctypes.c_uint8 * n)(*plan) if plan is not None else None
    return int(load().vlct_step_batch_until(n, g, a, dt_dev, next_dt_dev, status_dev, t_dev,
                                            t_end_dev,
                                            ctypes.cast(p, ctypes.c_void_p) if p is not None
                                            else None, ws, ws_bytes, stream))


def vlct_batch_tune(grids, states_in, states_out, dt_dev: int, ws: int, ws_bytes: int,
                    stream: int, reps: int = 3):
    """Returns (code, plan list) from the library's batch autotuner."""
    n = len(grids)
    g = (vlct_grid * n)(*grids)
    a = (vlct_state * n)(*states_in)
    b = (vlct_state * n)(*states_out)
    p = (ctypes.c_uint8 * n)()
    rc = int(load().vlct_batch_tune(n, g, a, b, dt_dev, ws, ws_bytes, stream, int(reps),
                                    ctypes.cast(p, ctypes.c_void_p)))
    return rc, [int(x) for x in p]


def vlct_strerror(code: int) -> str:
    return load().vlct_strerror(int(code)).decode()


def vlct_abi_version() -> int:
    return int(load().vlct_abi_version())


def vlct_step_observed(grid: vlct_grid, state_in: vlct_state, state_out: vlct_state, dt_dev: int,
                       next_dt_dev: int, status_dev: int, ws: int, ws_bytes: int, stream: int,
                       cb) -> int:
    """vlct_step that calls the Python callable cb(kernel, phase, stream)
    around each kernel launch of this call."""
    wrapped = vlct_launch_observer(lambda user, k, ph, st: cb(k, ph, st or 0))
    return int(load().vlct_step_observed(ctypes.byref(grid), ctypes.byref(state_in),
                                         ctypes.byref(state_out), dt_dev, next_dt_dev, status_dev,
                                         ws, ws_bytes, stream, wrapped, None))


def vlct_kernel_name(kernel: int) -> str:
    return load().vlct_kernel_name(int(kernel)).decode()
