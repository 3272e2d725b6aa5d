"""Helpers shared by the parity tests: the comparison metric, sampled-window
oracle evaluation for full-size runs, and GPU availability."""
from __future__ import annotations

import math
import os

import numpy as np

from paper_2402_05240_amd import inputs as I

FIELDS = I.FIELDS
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def gpu_available() -> bool:
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:  # pragma: no cover
        return False


def scales(g, s0):
    """Per-variable comparison scales of an initial state: rho -> mean rho,
    momenta -> mean rho * max signal speed, E -> mean E, face B -> mean |B|.
    They floor the denominator of the relative L1 metric so that fields that
    are tiny compared with their fluxes (momenta of a 1e-6 wave) are compared
    on the scale of the flow rather than on their own."""
    rho = s0["rho"]
    bcx = 0.5 * (s0["bx"][:, :, :-1] + s0["bx"][:, :, 1:])
    bcy = 0.5 * (s0["by"][:, :-1, :] + s0["by"][:, 1:, :])
    bcz = 0.5 * (s0["bz"][:-1, :, :] + s0["bz"][1:, :, :])
    b2 = bcx ** 2 + bcy ** 2 + bcz ** 2
    v2 = (s0["mx"] ** 2 + s0["my"] ** 2 + s0["mz"] ** 2) / rho ** 2
    p = (g.gamma - 1) * (s0["E"] - 0.5 * rho * v2 - 0.5 * b2)
    cmax = float(np.max(np.sqrt(v2) + np.sqrt((g.gamma * np.abs(p) + b2) / rho)))
    rbar = float(np.mean(rho))
    bbar = float(np.mean(np.sqrt(b2)))
    if bbar == 0.0:
        bbar = math.sqrt(float(np.mean(np.abs(p))))
    sc = {"rho": rbar, "E": float(np.mean(np.abs(s0["E"])))}
    for f in ("mx", "my", "mz"):
        sc[f] = rbar * cmax
    for f in ("bx", "by", "bz"):
        sc[f] = bbar
    return sc


def rel_l1(a, b, sc):
    """Per-variable relative L1 difference with scale floors."""
    out = {}
    for f in FIELDS:
        num = float(np.sum(np.abs(a[f] - b[f])))
        den = max(float(np.sum(np.abs(b[f]))), b[f].size * sc[f])
        out[f] = num / den
    return out


def max_abs_over_scale(a, b, sc):
    return {f: float(np.max(np.abs(a[f] - b[f]))) / sc[f] for f in FIELDS}


def window(g, s, center, h):
    """Sub-grid of (2h+1)^3 cells around `center` (i, j, k) taken from state s
    with the grid's own boundary mapping; on a periodic axis the window wraps,
    on an outflow axis it is shifted to stay inside the domain.  Returns the
    window grid (outflow on every axis), its state and the window index of the
    centre cell."""
    n = (g.nx, g.ny, g.nz)
    W = 2 * h + 1
    start, cw = [], []
    for d in range(3):
        if n[d] < W:
            raise ValueError("grid smaller than the window")
        if g.bc[d] == I.BC_PERIODIC:
            st = center[d] - h
        else:
            st = min(max(center[d] - h, 0), n[d] - W)
        start.append(st)
        cw.append(center[d] - st)
    ix = [(np.arange(W) + start[d]) % n[d] for d in range(3)]
    fx = [(np.arange(W + 1) + start[d]) % n[d] if g.bc[d] == I.BC_PERIODIC
          else np.arange(W + 1) + start[d] for d in range(3)]
    wg = I.Grid(W, W, W, g.dx, g.dy, g.dz, g.gamma, g.cfl, g.recon, (1, 1, 1))
    ws = {}
    for f in ("rho", "mx", "my", "mz", "E"):
        ws[f] = np.ascontiguousarray(s[f][np.ix_(ix[2], ix[1], ix[0])])
    ws["bx"] = np.ascontiguousarray(s["bx"][np.ix_(ix[2], ix[1], fx[0])])
    ws["by"] = np.ascontiguousarray(s["by"][np.ix_(ix[2], fx[1], ix[0])])
    ws["bz"] = np.ascontiguousarray(s["bz"][np.ix_(fx[2], ix[1], ix[0])])
    return wg, ws, tuple(cw)


def cell_values(g, s, c):
    """The 8 values owned by cell c = (i, j, k): 5 cell variables and its three
    low faces."""
    i, j, k = c
    return np.array([s["rho"][k, j, i], s["mx"][k, j, i], s["my"][k, j, i], s["mz"][k, j, i],
                     s["E"][k, j, i], s["bx"][k, j, i], s["by"][k, j, i], s["bz"][k, j, i]])


# a one-step result depends on cells within 4 of it (checked by a test); margin 2
WINDOW_HALF = 6
