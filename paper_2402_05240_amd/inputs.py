"""Seeded synthetic initial conditions for the VL+CT step.

This module builds inputs only: it holds none of the integrator's arithmetic
(no fluxes, reconstruction, Riemann solver or constrained transport). Both the
GPU library's callers and the CPU oracle take their inputs from here.

State layout (numpy float64, C order, x fastest), matching the C ABI:
  rho, mx, my, mz, E : (nz, ny, nx)
  bx                 : (nz, ny, nx+1)   face i-1/2 of cell i
  by                 : (nz, ny+1, nx)
  bz                 : (nz+1, ny, nx)
Coordinates: face i-1/2 sits at x = x0 + i*dx, cell i's centre at x0 + (i+1/2)*dx.

Workloads (the paper's own performance run is a slow magnetosonic linear wave,
Sec. 3.2; its accuracy suite is Sec. 3.1):
  * linear_wave  -- one MHD eigenmode on a periodic box (Sec. 3.1.1),
  * turbulence   -- decaying MHD turbulence from seeded Gaussian random fields,
  * blast        -- magnetised blast wave with outflow boundaries (Sec. 3.1.5),
  * uniform      -- a constant state (invariance checks).
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, Tuple

import numpy as np

FIELDS = ("rho", "mx", "my", "mz", "E", "bx", "by", "bz")

RECON_PCM = 1
RECON_PLMC = 2
RECON_PPMC = 3
RECON_PLMP = 4
RECON_PPMP = 5
BC_PERIODIC = 0
BC_OUTFLOW = 1


@dataclasses.dataclass
class Grid:
    """Mesh and run parameters handed to both the GPU library and the oracle."""

    nx: int
    ny: int
    nz: int
    dx: float
    dy: float
    dz: float
    gamma: float = 5.0 / 3.0
    cfl: float = 0.4
    recon: int = RECON_PLMC
    bc: Tuple[int, int, int] = (BC_PERIODIC, BC_PERIODIC, BC_PERIODIC)

    @property
    def shape(self) -> Tuple[int, int, int]:
        return (self.nz, self.ny, self.nx)

    @property
    def ncells(self) -> int:
        return self.nx * self.ny * self.nz

    def field_shape(self, name: str) -> Tuple[int, int, int]:
        nz, ny, nx = self.shape
        if name == "bx":
            return (nz, ny, nx + 1)
        if name == "by":
            return (nz, ny + 1, nx)
        if name == "bz":
            return (nz + 1, ny, nx)
        return (nz, ny, nx)


State = Dict[str, np.ndarray]


def empty_state(g: Grid) -> State:
    return {f: np.zeros(g.field_shape(f), dtype=np.float64) for f in FIELDS}


def copy_state(s: State) -> State:
    return {f: np.array(s[f], dtype=np.float64, copy=True) for f in FIELDS}


def _cell_energy(g: Grid, rho, vx, vy, vz, p, bx, by, bz) -> np.ndarray:
    """Total energy from primitives with the cell-centred field taken as the
    average of the two face values (the state definition of Sec. 2.1)."""
    bcx = 0.5 * (bx[:, :, :-1] + bx[:, :, 1:])
    bcy = 0.5 * (by[:, :-1, :] + by[:, 1:, :])
    bcz = 0.5 * (bz[:-1, :, :] + bz[1:, :, :])
    return (p / (g.gamma - 1.0) + 0.5 * rho * (vx * vx + vy * vy + vz * vz)
            + 0.5 * (bcx * bcx + bcy * bcy + bcz * bcz))


def _periodic_face_copy(g: Grid, s: State) -> None:
    """On periodic axes the duplicated last face plane equals the first."""
    if g.bc[0] == BC_PERIODIC:
        s["bx"][:, :, -1] = s["bx"][:, :, 0]
    if g.bc[1] == BC_PERIODIC:
        s["by"][:, -1, :] = s["by"][:, 0, :]
    if g.bc[2] == BC_PERIODIC:
        s["bz"][-1, :, :] = s["bz"][0, :, :]


# --------------------------------------------------------------------------
# uniform state
# --------------------------------------------------------------------------

def uniform(n=(16, 16, 16), rho=1.0, v=(0.0, 0.0, 0.0), p=0.6, b=(1.0, 0.0, 0.0),
            gamma=5.0 / 3.0, cfl=0.4, recon=RECON_PLMC, bc=(0, 0, 0),
            length=(1.0, 1.0, 1.0)) -> Tuple[Grid, State]:
    nx, ny, nz = n
    g = Grid(nx, ny, nz, length[0] / nx, length[1] / ny, length[2] / nz, gamma, cfl,
             recon, tuple(bc))
    s = empty_state(g)
    s["rho"][:] = rho
    s["mx"][:] = rho * v[0]
    s["my"][:] = rho * v[1]
    s["mz"][:] = rho * v[2]
    s["bx"][:] = b[0]
    s["by"][:] = b[1]
    s["bz"][:] = b[2]
    s["E"][:] = p / (gamma - 1.0) + 0.5 * rho * (v[0] ** 2 + v[1] ** 2 + v[2] ** 2) \
        + 0.5 * (b[0] ** 2 + b[1] ** 2 + b[2] ** 2)
    return g, s


# --------------------------------------------------------------------------
# linear MHD waves (Sec. 3.1.1)
# --------------------------------------------------------------------------

WAVES = ("fast", "alfven", "slow", "contact")


def primitive_jacobian(rho, u, v, w, p, by, bz, bn, gamma) -> np.ndarray:
    """Coefficient matrix A of the 1D ideal-MHD system dW/dt + A dW/dx = 0 in
    W = (rho, u, v, w, P, B_t1, B_t2), written out from the equations of
    Sec. 2.1 (mu0 = 1, B_n constant). Used only to set up eigenmode ICs."""
    A = np.zeros((7, 7))
    A[0, 0] = u
    A[0, 1] = rho
    A[1, 1] = u
    A[1, 4] = 1.0 / rho
    A[1, 5] = by / rho
    A[1, 6] = bz / rho
    A[2, 2] = u
    A[2, 5] = -bn / rho
    A[3, 3] = u
    A[3, 6] = -bn / rho
    A[4, 1] = gamma * p
    A[4, 4] = u
    A[5, 1] = by
    A[5, 2] = -bn
    A[5, 5] = u
    A[6, 1] = bz
    A[6, 3] = -bn
    A[6, 6] = u
    return A


def conserved_eigenmode(wave: str, rho, vel, p, b, gamma) -> Tuple[np.ndarray, float]:
    """Right-going eigenvector of `wave` in conserved variables
    (rho, m_n, m_t1, m_t2, E, B_t1, B_t2) for a background given in the sweep
    frame, normalised to unit max-norm with its largest entry positive, and
    the wave's phase speed. Computed numerically from the primitive Jacobian."""
    u, v, w = vel
    bn, by, bz = b
    A = primitive_jacobian(rho, u, v, w, p, by, bz, bn, gamma)
    lam, vec = np.linalg.eig(A)
    lam = lam.real
    vec = vec.real
    a2 = gamma * p / rho
    b2 = bn * bn + by * by + bz * bz
    disc = math.sqrt(max((a2 + b2 / rho) ** 2 - 4.0 * a2 * bn * bn / rho, 0.0))
    cf = math.sqrt(0.5 * (a2 + b2 / rho + disc))
    cs = math.sqrt(max(0.5 * (a2 + b2 / rho - disc), 0.0))
    ca = abs(bn) / math.sqrt(rho)
    target = {"fast": u + cf, "alfven": u + ca, "slow": u + cs, "contact": u}[wave]
    m = int(np.argmin(np.abs(lam - target)))
    if abs(lam[m] - target) > 1e-8 * max(1.0, abs(target)):
        raise ValueError("eigenvalue for %s wave not found" % wave)
    if np.sum(np.abs(lam - target) < 1e-8 * max(1.0, abs(target))) != 1:
        raise ValueError("%s wave speed is degenerate for this background" % wave)
    rp = vec[:, m]
    # dU/dW for U = (rho, rho u, rho v, rho w, E, B_t1, B_t2)
    J = np.zeros((7, 7))
    J[0, 0] = 1.0
    J[1, 0], J[1, 1] = u, rho
    J[2, 0], J[2, 2] = v, rho
    J[3, 0], J[3, 3] = w, rho
    J[4, :] = [0.5 * (u * u + v * v + w * w), rho * u, rho * v, rho * w,
               1.0 / (gamma - 1.0), by, bz]
    J[5, 5] = 1.0
    J[6, 6] = 1.0
    rc = J @ rp
    rc = rc / np.max(np.abs(rc))
    if rc[np.argmax(np.abs(rc))] < 0:
        rc = -rc
    return rc, target


def linear_wave(n=(32, 32, 32), wave="fast", amp=1e-6, axis=0, gamma=5.0 / 3.0,
                b_sweep=(1.0, math.sqrt(2.0), 0.5), rho=1.0, p=None, vn=0.0,
                recon=RECON_PLMC, cfl=0.4) -> Tuple[Grid, State, float]:
    """Eigenmode q = q_bar + amp * R_w * sin(2 pi s) along `axis` (0, 1, 2) on the
    unit periodic box (Sec. 3.1.1); the background field and velocity are given in
    the sweep frame (n, t1, t2) of that axis, so the same 1D problem can be run
    along every axis.  Returns (grid, state, period)."""
    if p is None:
        p = 1.0 / gamma
    if wave == "contact" and vn == 0.0:
        vn = 1.0
    nx, ny, nz = n
    g = Grid(nx, ny, nz, 1.0 / nx, 1.0 / ny, 1.0 / nz, gamma, cfl, recon, (0, 0, 0))
    rc, speed = conserved_eigenmode(wave, rho, (vn, 0.0, 0.0), p, b_sweep, gamma)
    period = 1.0 / abs(speed)
    nd = (nx, ny, nz)[axis]
    xc = (np.arange(nd) + 0.5) / nd
    ph = np.sin(2.0 * np.pi * xc)
    # background conserved sweep-frame state
    bn, bt1, bt2 = b_sweep
    e_bar = p / (gamma - 1.0) + 0.5 * rho * vn * vn + 0.5 * (bn * bn + bt1 * bt1 + bt2 * bt2)
    qbar = np.array([rho, rho * vn, 0.0, 0.0, e_bar, bt1, bt2])
    q = qbar[:, None] + amp * rc[:, None] * ph[None, :]   # (7, nd)
    t1, t2 = (axis + 1) % 3, (axis + 2) % 3
    s = empty_state(g)

    def along(vals, shape, ax):
        # broadcast a 1D profile along lab axis ax (0 = x) onto array shape (z, y, x)
        sh = [1, 1, 1]
        sh[2 - ax] = len(vals)
        return np.broadcast_to(vals.reshape(sh), shape).copy()

    shp = g.shape
    s["rho"] = along(q[0], shp, axis)
    mom = {axis: q[1], t1: q[2], t2: q[3]}
    s["mx"] = along(mom[0], shp, axis)
    s["my"] = along(mom[1], shp, axis)
    s["mz"] = along(mom[2], shp, axis)
    s["E"] = along(q[4], shp, axis)
    bl = {axis: np.full(nd, bn), t1: q[5], t2: q[6]}
    for d, name in enumerate(("bx", "by", "bz")):
        fs = g.field_shape(name)
        if d == axis:
            s[name] = np.full(fs, bn)
        else:
            s[name] = along(bl[d], fs, axis)
    return g, s, period


def oblique_wave(n=(32, 32, 1), wave="fast", amp=1e-6, kvec=(1, 1, 0), gamma=5.0 / 3.0,
                 b_sweep=(1.0, math.sqrt(2.0), 0.5), rho=1.0, p=None, vn=0.0,
                 recon=RECON_PLMC, cfl=0.4) -> Tuple[Grid, State, float]:
    """Eigenmode travelling along the integer wavevector kvec of the periodic
    unit box (a grid-oblique version of Sec. 3.1.1's linear waves).  The
    background field is (b_n, b_t1, b_t2) in the frame (k/|k|, t1, t2); the field
    perturbation is set through an edge-centred vector potential so the initial
    face field is divergence-free to rounding.  Returns (grid, state, period)."""
    if p is None:
        p = 1.0 / gamma
    if wave == "contact" and vn == 0.0:
        vn = 1.0
    nx, ny, nz = n
    g = Grid(nx, ny, nz, 1.0 / nx, 1.0 / ny, 1.0 / nz, gamma, cfl, recon, (0, 0, 0))
    kv = np.array(kvec, dtype=float)
    kn = kv / np.linalg.norm(kv)
    trial = np.array([0.0, 0.0, 1.0]) if abs(kn[2]) < 0.9 else np.array([1.0, 0.0, 0.0])
    t2 = trial - kn * (trial @ kn)
    t2 /= np.linalg.norm(t2)
    t1 = np.cross(t2, kn)
    rc, speed = conserved_eigenmode(wave, rho, (vn, 0.0, 0.0), p, b_sweep, gamma)
    wavelength = 1.0 / np.linalg.norm(kv)
    period = wavelength / abs(speed)
    bn, bt1, bt2 = b_sweep
    bbar = bn * kn + bt1 * t1 + bt2 * t2
    K = 2.0 * np.pi * kv

    def coords(off):
        x = (np.arange(nx) + off[0]) / nx
        y = (np.arange(ny) + off[1]) / ny
        z = (np.arange(nz) + off[2]) / nz
        return K[0] * x[None, None, :] + K[1] * y[None, :, None] + K[2] * z[:, None, None]

    th = coords((0.5, 0.5, 0.5))
    sn = np.sin(th)
    s = empty_state(g)
    e_bar = p / (gamma - 1.0) + 0.5 * rho * vn * vn + 0.5 * float(bbar @ bbar)
    s["rho"] = rho + amp * rc[0] * sn
    mvec_bar = rho * vn * kn
    mvec = amp * (rc[1] * kn + rc[2] * t1 + rc[3] * t2)
    s["mx"] = mvec_bar[0] + mvec[0] * sn
    s["my"] = mvec_bar[1] + mvec[1] * sn
    s["mz"] = mvec_bar[2] + mvec[2] * sn
    s["E"] = e_bar + amp * rc[4] * sn
    bvec = amp * (rc[5] * t1 + rc[6] * t2)
    avec = np.cross(K, bvec) / float(K @ K)      # curl(a cos(K.x)) = bvec sin(K.x)
    ax = avec[0] * np.cos(coords((0.5, 0.0, 0.0)))
    ay = avec[1] * np.cos(coords((0.0, 0.5, 0.0)))
    az = avec[2] * np.cos(coords((0.0, 0.0, 0.5)))
    bxf, byf, bzf = curl_edge_potential(g, ax, ay, az)
    s["bx"] = bbar[0] + bxf
    s["by"] = bbar[1] + byf
    s["bz"] = bbar[2] + bzf
    _periodic_face_copy(g, s)
    return g, s, period


def field_loop_2d(n=32, amp=1e-3, radius=0.3, v=(2.0, 1.0, 0.0), rho=1.0, p=1.0,
                  gamma=5.0 / 3.0, recon=RECON_PLMC, cfl=0.4) -> Tuple[Grid, State]:
    """Advected field loop (the 2D form of Sec. 3.1.3's test): a cylinder of
    field lines, A_z = amp (R - r) inside r < R, carried by a uniform flow
    across the periodic unit square (one cell thick in z)."""
    g, s = uniform((n, n, 1), rho=rho, v=v, p=p, b=(0.0, 0.0, 0.0), gamma=gamma, cfl=cfl,
                   recon=recon, bc=(0, 0, 0), length=(1.0, 1.0, 1.0 / n))
    x = -0.5 + np.arange(n) / n
    y = -0.5 + np.arange(n) / n
    r = np.sqrt(x[None, :] ** 2 + y[:, None] ** 2)
    az = np.where(r < radius, amp * (radius - r), 0.0)[None, :, :]
    zero = np.zeros((1, n, n))
    s["bx"], s["by"], s["bz"] = curl_edge_potential(g, zero, zero, az)
    s["E"] = _cell_energy(g, s["rho"], s["mx"] / rho, s["my"] / rho, s["mz"] / rho, p,
                          s["bx"], s["by"], s["bz"])
    return g, s


# --------------------------------------------------------------------------
# circularly polarised Alfven wave (Sec. 3.1.2), Orszag-Tang vortex (Sec. 3.1.6),
# tilted spherical field loop (Sec. 3.1.3)
# --------------------------------------------------------------------------

def _centres(g: Grid, origin=(0.0, 0.0, 0.0), off=(0.5, 0.5, 0.5)):
    """Physical coordinates (x, y, z) broadcastable to (nz, ny, nx) of the points
    at index offsets `off` (0.5 = cell centre, 0 = lower face)."""
    x = origin[0] + (np.arange(g.nx) + off[0]) * g.dx
    y = origin[1] + (np.arange(g.ny) + off[1]) * g.dy
    z = origin[2] + (np.arange(g.nz) + off[2]) * g.dz
    return x[None, None, :], y[None, :, None], z[:, None, None]


def cpaw(N=16, standing=False, amp=0.1, wavelength=1.0, gamma=5.0 / 3.0, recon=RECON_PLMC,
         cfl=0.4) -> Tuple[Grid, State, float]:
    """Circularly polarised Alfven wave on the periodic 3.0 x 1.5 x 1.5 box at
    2N x N x N.  In the wave frame rho = 1, P = 0.1, v = (v_par, A sin phi,
    A cos phi), B = (1, A sin phi, A cos phi), phi = 2 pi x1 / lambda, with v_par
    = 0 (travelling) or -1 (standing).  The wave frame is the lab frame rotated
    by sin(alpha) = 2/3, sin(beta) = 2/sqrt(5), so the wave vector
    (1/3, 2/3, 2/3) fits the box once along every axis.  The field perturbation
    comes from an edge-centred vector potential.  Returns (grid, state, period)."""
    g = Grid(2 * N, N, N, 3.0 / (2 * N), 1.5 / N, 1.5 / N, gamma, cfl, recon, (0, 0, 0))
    sa, ca = 2.0 / 3.0, math.sqrt(5.0) / 3.0
    sb, cb = 2.0 / math.sqrt(5.0), 1.0 / math.sqrt(5.0)
    e1 = np.array([ca * cb, ca * sb, sa])
    e2 = np.array([-sb, cb, 0.0])
    e3 = np.array([-sa * cb, -sa * sb, ca])
    kw = 2.0 * math.pi / wavelength

    def phase(off):
        x, y, z = _centres(g, off=off)
        return kw * (e1[0] * x + e1[1] * y + e1[2] * z)
    ph = phase((0.5, 0.5, 0.5))
    rho, p, b1 = 1.0, 0.1, 1.0
    vpar = -1.0 if standing else 0.0
    s = empty_state(g)
    v = [vpar * e1[c] + amp * (np.sin(ph) * e2[c] + np.cos(ph) * e3[c]) for c in range(3)]
    s["rho"] = np.full(g.shape, rho)
    s["mx"], s["my"], s["mz"] = rho * v[0], rho * v[1], rho * v[2]
    a = amp / kw       # curl of a (sin phi e2 + cos phi e3) = A (sin phi e2 + cos phi e3)
    ax = a * (np.sin(phase((0.5, 0.0, 0.0))) * e2[0] + np.cos(phase((0.5, 0.0, 0.0))) * e3[0])
    ay = a * (np.sin(phase((0.0, 0.5, 0.0))) * e2[1] + np.cos(phase((0.0, 0.5, 0.0))) * e3[1])
    az = a * (np.sin(phase((0.0, 0.0, 0.5))) * e2[2] + np.cos(phase((0.0, 0.0, 0.5))) * e3[2])
    ax, ay, az = (np.broadcast_to(q, g.shape).copy() for q in (ax, ay, az))
    bxf, byf, bzf = curl_edge_potential(g, ax, ay, az)
    s["bx"], s["by"], s["bz"] = bxf + b1 * e1[0], byf + b1 * e1[1], bzf + b1 * e1[2]
    _periodic_face_copy(g, s)
    s["E"] = _cell_energy(g, s["rho"], v[0], v[1], v[2], p, s["bx"], s["by"], s["bz"])
    return g, s, wavelength / (b1 / math.sqrt(rho))


def orszag_tang(n=(64, 64, 2), gamma=5.0 / 3.0, recon=RECON_PLMC, cfl=0.4) -> Tuple[Grid, State]:
    """Orszag-Tang vortex on the periodic unit box (z-independent):
    rho = 25/(36 pi), P = 5/(12 pi), v = (sin 2 pi y, -sin 2 pi x, 0) and
    A_z = B0/(4 pi) (cos 4 pi x + 2 cos 2 pi y) with B0 = 1/sqrt(4 pi)."""
    nx, ny, nz = n
    g = Grid(nx, ny, nz, 1.0 / nx, 1.0 / ny, 1.0 / nz, gamma, cfl, recon, (0, 0, 0))
    rho, p = 25.0 / (36.0 * math.pi), 5.0 / (12.0 * math.pi)
    b0 = 1.0 / math.sqrt(4.0 * math.pi)
    x, y, _ = _centres(g)
    vx = np.broadcast_to(np.sin(2.0 * math.pi * y), g.shape).copy()
    vy = np.broadcast_to(-np.sin(2.0 * math.pi * x), g.shape).copy()
    vz = np.zeros(g.shape)
    xe, ye, _ = _centres(g, off=(0.0, 0.0, 0.5))
    az = np.broadcast_to(b0 / (4.0 * math.pi) * (np.cos(4.0 * math.pi * xe)
                                                 + 2.0 * np.cos(2.0 * math.pi * ye)),
                         g.shape).copy()
    zero = np.zeros(g.shape)
    s = empty_state(g)
    s["rho"] = np.full(g.shape, rho)
    s["mx"], s["my"], s["mz"] = rho * vx, rho * vy, rho * vz
    s["bx"], s["by"], s["bz"] = curl_edge_potential(g, zero, zero, az)
    s["E"] = _cell_energy(g, s["rho"], vx, vy, vz, p, s["bx"], s["by"], s["bz"])
    return g, s


def field_loop_3d(N=16, amp=1e-3, radius=0.3, v=(1.0, 1.0, 2.0), rho=1.0, p=1.0,
                  gamma=5.0 / 3.0, recon=RECON_PLMC, cfl=0.4) -> Tuple[Grid, State]:
    """Tilted spherical field loop: A_y = A_z = amp (R - r) inside r < R (r from
    the box centre, A_x = 0), carried by v = (1, 1, 2) across the periodic
    1 x 1 x 2 box centred at 0 on N x N x 2N cells (one period every unit of
    time)."""
    g = Grid(N, N, 2 * N, 1.0 / N, 1.0 / N, 1.0 / N, gamma, cfl, recon, (0, 0, 0))
    org = (-0.5, -0.5, -1.0)

    def pot(off):
        x, y, z = _centres(g, origin=org, off=off)
        r = np.sqrt(x * x + y * y + z * z)
        return np.where(r < radius, amp * (radius - r), 0.0)
    ax = np.zeros(g.shape)
    ay = np.broadcast_to(pot((0.0, 0.5, 0.0)), g.shape).copy()
    az = np.broadcast_to(pot((0.0, 0.0, 0.5)), g.shape).copy()
    s = empty_state(g)
    s["rho"] = np.full(g.shape, rho)
    s["mx"], s["my"], s["mz"] = (np.full(g.shape, rho * v[c]) for c in range(3))
    s["bx"], s["by"], s["bz"] = curl_edge_potential(g, ax, ay, az)
    s["E"] = _cell_energy(g, s["rho"], v[0], v[1], v[2], p, s["bx"], s["by"], s["bz"])
    return g, s


# --------------------------------------------------------------------------
# decaying MHD turbulence
# --------------------------------------------------------------------------

KMAX = 4


def _random_modes(rng: np.random.Generator):
    """Complex Gaussian coefficients on integer wavevectors 1 <= |k| <= KMAX with
    amplitude |k|^-2 (shell spectrum E(k) ~ k^-2), drawn in a fixed order so the
    continuous field does not depend on the grid resolution."""
    ks = []
    rng_k = np.arange(-KMAX, KMAX + 1)
    for kx in rng_k:
        for ky in rng_k:
            for kz in range(0, KMAX + 1):
                ks.append((kx, ky, kz))
    ks = np.array(ks)
    re = rng.standard_normal(len(ks))
    im = rng.standard_normal(len(ks))
    kk = np.sqrt((ks ** 2).sum(axis=1))
    keep = (kk >= 1.0) & (kk <= KMAX)
    # half-space kz >= 0; drop the redundant half of the kz = 0 plane
    half = (ks[:, 2] > 0) | (ks[:, 1] > 0) | ((ks[:, 1] == 0) & (ks[:, 0] > 0))
    keep &= half
    amp = np.where(keep, 1.0 / np.maximum(kk, 1.0) ** 2, 0.0)
    return ks[keep], (re + 1j * im)[keep] * amp[keep]


def _eval_modes(ks, coef, n, offset) -> np.ndarray:
    """Real field sum_k Re(c_k exp(2 pi i k.x)) sampled at x_d = (idx_d + offset_d)/n_d
    on an (nz, ny, nx) grid of the unit box, via one complex inverse FFT.  Needs
    n_d >= 2 KMAX + 1 so that no retained mode aliases."""
    nx, ny, nz = n
    if min(n) < 2 * KMAX + 1:
        raise ValueError("turbulence grid needs at least %d cells per axis" % (2 * KMAX + 1))
    spec = np.zeros((nz, ny, nx), dtype=np.complex128)
    ox, oy, oz = offset
    for (kx, ky, kz), c in zip(ks, coef):
        ph = np.exp(2j * np.pi * (kx * ox / nx + ky * oy / ny + kz * oz / nz))
        spec[kz % nz, ky % ny, kx % nx] += c * ph
    return np.fft.ifftn(spec).real * float(nx * ny * nz)


def turbulence(n=(256, 256, 256), seed_v=2402, seed_a=5240, mach=1.0, beta=1.0,
               db_rms=0.1, gamma=5.0 / 3.0, recon=RECON_PLMC, cfl=0.4) -> Tuple[Grid, State]:
    """Decaying MHD turbulence (see turbulence_potential)."""
    g, s, _, _ = turbulence_potential(n, seed_v, seed_a, mach, beta, db_rms, gamma, recon, cfl)
    return g, s


def turbulence_potential(n=(256, 256, 256), seed_v=2402, seed_a=5240, mach=1.0, beta=1.0,
                         db_rms=0.1, gamma=5.0 / 3.0, recon=RECON_PLMC, cfl=0.4):
    """Decaying MHD turbulence on the periodic unit box: rho = 1, sound speed 1
    (P = 1/gamma), velocity a Gaussian random field with E(k) ~ k^-2 on
    1 <= |k| <= 4 scaled to rms |v| = mach, uniform B_x with plasma beta `beta`
    plus a divergence-free perturbation B = curl A of an edge-centred random vector
    potential, scaled to rms |dB_cc| = db_rms * B_x0.

    Returns (grid, state, A, b0): the face field of the state is
    b0 + curl_h A with A = (ax, ay, az) the scaled edge potential (cell-shaped
    arrays, ax at (i, j-1/2, k-1/2) and cyclically) and b0 = (B_x0, 0, 0)."""
    nx, ny, nz = n
    g = Grid(nx, ny, nz, 1.0 / nx, 1.0 / ny, 1.0 / nz, gamma, cfl, recon, (0, 0, 0))
    rho = 1.0
    p = rho * 1.0 / gamma
    bx0 = math.sqrt(2.0 * p / beta)
    rng_v = np.random.default_rng(seed_v)
    vel = []
    for _ in range(3):
        ks, coef = _random_modes(rng_v)
        vel.append(_eval_modes(ks, coef, n, (0.5, 0.5, 0.5)))
    vx, vy, vz = vel
    for f in (vx, vy, vz):
        f -= f.mean()
    vrms = math.sqrt(float(np.mean(vx * vx + vy * vy + vz * vz)))
    vx *= mach / vrms
    vy *= mach / vrms
    vz *= mach / vrms

    rng_a = np.random.default_rng(seed_a)
    offs = ((0.5, 0.0, 0.0), (0.0, 0.5, 0.0), (0.0, 0.0, 0.5))
    pot = []
    for d in range(3):
        ks, coef = _random_modes(rng_a)
        pot.append(_eval_modes(ks, coef, n, offs[d]))
    bxf, byf, bzf = curl_edge_potential(g, *pot)
    # scale the perturbation
    bcx = 0.5 * (bxf[:, :, :-1] + bxf[:, :, 1:])
    bcy = 0.5 * (byf[:, :-1, :] + byf[:, 1:, :])
    bcz = 0.5 * (bzf[:-1, :, :] + bzf[1:, :, :])
    brms = math.sqrt(float(np.mean(bcx * bcx + bcy * bcy + bcz * bcz)))
    sc = db_rms * bx0 / brms
    s = empty_state(g)
    s["bx"] = bx0 + sc * bxf
    s["by"] = sc * byf
    s["bz"] = sc * bzf
    _periodic_face_copy(g, s)
    s["rho"][:] = rho
    s["mx"] = rho * vx
    s["my"] = rho * vy
    s["mz"] = rho * vz
    s["E"] = _cell_energy(g, s["rho"], vx, vy, vz, p, s["bx"], s["by"], s["bz"])
    return g, s, [sc * a for a in pot], (bx0, 0.0, 0.0)


def curl_edge_potential(g: Grid, ax: np.ndarray, ay: np.ndarray, az: np.ndarray):
    """Face fields B = curl A of an edge-centred vector potential on a periodic
    grid: ax[k,j,i] at (i, j-1/2, k-1/2), ay at (i-1/2, j, k-1/2), az at
    (i-1/2, j-1/2, k).  The discrete divergence of the result vanishes up to
    rounding.  Returns (bx, by, bz) in the state's face layout."""
    dx, dy, dz = g.dx, g.dy, g.dz

    def fwd(a, axis):  # a(idx + 1) - a(idx), periodic
        return np.roll(a, -1, axis=axis) - a

    bx = fwd(az, 1) / dy - fwd(ay, 0) / dz
    by = fwd(ax, 0) / dz - fwd(az, 2) / dx
    bz = fwd(ay, 2) / dx - fwd(ax, 1) / dy
    bxf = np.concatenate([bx, bx[:, :, :1]], axis=2)
    byf = np.concatenate([by, by[:, :1, :]], axis=1)
    bzf = np.concatenate([bz, bz[:1, :, :]], axis=0)
    return bxf, byf, bzf


# --------------------------------------------------------------------------
# magnetised blast wave (Sec. 3.1.5)
# --------------------------------------------------------------------------

def blast(n=(512, 512, 512), gamma=5.0 / 3.0, p_in=10.0, p_out=0.1, r0=0.1,
          b0=10.0 / math.sqrt(4.0 * math.pi), recon=RECON_PPMC, cfl=0.4,
          length=(1.0, 1.0, 1.0)) -> Tuple[Grid, State]:
    """Blast wave in a magnetised medium on the box [-L/2, L/2)^3 with outflow
    boundaries: rho = 1, v = 0, P = p_out outside and p_in inside a sphere of
    radius r0 (cell centres), uniform B = b0 (1, 1, 0)/sqrt(2)."""
    nx, ny, nz = n
    g = Grid(nx, ny, nz, length[0] / nx, length[1] / ny, length[2] / nz, gamma, cfl, recon,
             (BC_OUTFLOW, BC_OUTFLOW, BC_OUTFLOW))
    x = -0.5 * length[0] + (np.arange(nx) + 0.5) * g.dx
    y = -0.5 * length[1] + (np.arange(ny) + 0.5) * g.dy
    z = -0.5 * length[2] + (np.arange(nz) + 0.5) * g.dz
    r2 = z[:, None, None] ** 2 + y[None, :, None] ** 2 + x[None, None, :] ** 2
    p = np.where(r2 < r0 * r0, p_in, p_out)
    s = empty_state(g)
    bxv = b0 / math.sqrt(2.0)
    s["rho"][:] = 1.0
    s["bx"][:] = bxv
    s["by"][:] = bxv
    s["bz"][:] = 0.0
    s["E"] = p / (gamma - 1.0) + 0.5 * (2.0 * bxv * bxv)
    return g, s


# --------------------------------------------------------------------------
# MHD Riemann problems (Sec. 3.1.4, Table "Riemann Problem Initial Conditions")
# --------------------------------------------------------------------------

def riemann(left, right, bn, gamma, n=128, axis=0, flip=False, transverse=4,
            recon=RECON_PPMC, cfl=0.4) -> Tuple[Grid, State]:
    """A 1D Riemann problem on the unit box along `axis` with the interface at
    the middle and outflow boundaries along it (periodic across).  `left` and
    `right` are sweep-frame primitives (rho, P, v_n, v_t1, v_t2, B_t1, B_t2); B_n
    is the same on both sides.  flip=True mirrors the problem (states swapped,
    normal vector components negated)."""
    L = np.array(left, dtype=float)
    R = np.array(right, dtype=float)
    if flip:
        L, R = R.copy(), L.copy()
        L[2] = -L[2]
        R[2] = -R[2]
        bn = -bn
    shape = [transverse, transverse, transverse]
    shape[axis] = n
    nx, ny, nz = shape
    bc = [BC_PERIODIC] * 3
    bc[axis] = BC_OUTFLOW
    g = Grid(nx, ny, nz, 1.0 / nx, 1.0 / ny, 1.0 / nz, gamma, cfl, recon, tuple(bc))
    xc = (np.arange(n) + 0.5) / n
    left_side = xc < 0.5
    prof = np.where(left_side[:, None], L[None, :], R[None, :])   # (n, 7)
    t1, t2 = (axis + 1) % 3, (axis + 2) % 3
    s = empty_state(g)

    def along(vals, shp):
        sh = [1, 1, 1]
        sh[2 - axis] = len(vals)
        return np.broadcast_to(vals.reshape(sh), shp).copy()
    rho, p = prof[:, 0], prof[:, 1]
    vel = {axis: prof[:, 2], t1: prof[:, 3], t2: prof[:, 4]}
    bt = {t1: prof[:, 5], t2: prof[:, 6]}
    s["rho"] = along(rho, g.shape)
    for d, name in enumerate(("mx", "my", "mz")):
        s[name] = along(rho * vel[d], g.shape)
    for d, name in enumerate(("bx", "by", "bz")):
        fs = g.field_shape(name)
        s[name] = np.full(fs, bn) if d == axis else along(bt[d], fs)
    ke = 0.5 * rho * (prof[:, 2] ** 2 + prof[:, 3] ** 2 + prof[:, 4] ** 2)
    me = 0.5 * (bn * bn + prof[:, 5] ** 2 + prof[:, 6] ** 2)
    s["E"] = along(p / (gamma - 1.0) + ke + me, g.shape)
    return g, s


# --------------------------------------------------------------------------
# ensembles of independent small runs (batched stepping)
# --------------------------------------------------------------------------

def ensemble(count=64, seed=2402, nmin=16, nmax=96, recon=RECON_PLMC, cfl=0.4):
    """`count` independent periodic linear-wave problems: sizes drawn uniformly
    from nmin..nmax per axis (non-cubic), gamma uniform in [1.4, 5/3], the fast,
    slow or Alfven family, a random grid-oblique direction (integer wavevector
    with components in {-1, 0, 1}), amplitude log-uniform in [1e-6, 1e-4].
    Returns [(grid, state, period)]."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        n = tuple(int(v) for v in rng.integers(nmin, nmax + 1, size=3))
        gamma = float(rng.uniform(1.4, 5.0 / 3.0))
        wave = ("fast", "slow", "alfven")[int(rng.integers(0, 3))]
        while True:
            kvec = tuple(int(v) for v in rng.integers(-1, 2, size=3))
            if any(kvec):
                break
        amp = float(10.0 ** rng.uniform(-6.0, -4.0))
        out.append(oblique_wave(n, wave, amp=amp, kvec=kvec, gamma=gamma, recon=recon, cfl=cfl))
    return out


# --------------------------------------------------------------------------
# named workloads
# --------------------------------------------------------------------------

def workload(name: str, scale: int = None):
    """Named synthetic workloads.  `scale` overrides the cube edge length."""
    if name == "linear_fast_32":
        m = scale or 32
        g, s, period = linear_wave((m, m, m), "fast")
        return g, s
    if name == "turbulence_plmc_256":
        m = scale or 256
        return turbulence((m, m, m), recon=RECON_PLMC)
    if name == "turbulence_ppmc_256":
        m = scale or 256
        return turbulence((m, m, m), recon=RECON_PPMC)
    if name == "blast_ppmc_512":
        m = scale or 512
        return blast((m, m, m))
    raise KeyError(name)
