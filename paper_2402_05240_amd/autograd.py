"""Differentiable VL+CT rollouts on the GPU.

torch.autograd.Function wrappers around the library's step (vlct_step), its
adjoint (vlct_step_adjoint) and the vector-potential map B = curl_h A
(vlct_curl_potential and its transpose).  Every computation runs in
libvlct.so; this module only orders the calls and holds the checkpoints.

Step sizes are parameters of the rollout, not differentiated: a rollout
either takes a list of device dt words or records the CFL chain of its
forward pass (each step's dt is the previous step's next-dt output) and
reuses exactly those values when it recomputes states for the backward pass.

Memory: a rollout of N steps keeps its input and one state every `segment`
steps (default ceil(sqrt(N))); the backward pass recomputes one segment at a
time from its checkpoint with taped steps (vlct_step_taped: the half-step
state and the faces' upwind sides of each step, so the adjoint need not
recompute the fluxes), so at most about sqrt(N) states and sqrt(N) tapes are
alive.
"""
from __future__ import annotations

import math
from typing import List, Optional, Sequence, Tuple

from . import vlct
from .inputs import FIELDS, Grid


def _torch():
    import torch
    return torch


Fields = Tuple["torch.Tensor", ...]  # noqa: F821  (8 device tensors in FIELDS order)


class Simulator:
    """Device workspaces for forward steps, adjoints and the curl of one
    periodic grid; all calls go to torch's current stream."""

    def __init__(self, grid: Grid, device: str = "cuda:0"):
        torch = _torch()
        if any(int(b) != vlct.VLCT_BC_PERIODIC for b in grid.bc):
            raise ValueError("differentiable rollouts need periodic boundaries")
        self.grid = grid
        self.device = device
        self.cg = vlct.make_grid(grid)
        self.ws_step_bytes = vlct.vlct_workspace_bytes(self.cg)
        self.ws_adj_bytes = vlct.vlct_adjoint_workspace_bytes(self.cg)
        if not self.ws_step_bytes or not self.ws_adj_bytes:
            raise ValueError("invalid grid descriptor")
        self.ws_step = torch.empty(self.ws_step_bytes, dtype=torch.uint8, device=device)
        self._ws_adj = None
        self._ws_adj_taped = None
        self.tape_bytes = vlct.vlct_tape_bytes(self.cg)
        self.ws_adj_taped_bytes = vlct.vlct_adjoint_taped_workspace_bytes(self.cg)
        self.status = torch.zeros(1, dtype=torch.int32, device=device)

    def _stream(self) -> int:
        return _torch().cuda.current_stream().cuda_stream

    def raise_on_status(self, where: str) -> None:
        """One host read of the status word the steps accumulate: a floor or a
        non-finite value makes the loss and its gradient those of the floored
        branch (or meaningless), so a rollout reports it instead of returning
        them silently."""
        bits = int(self.status.item())
        if bits:
            names = [n for b, n in ((vlct.VLCT_STATUS_PRESSURE_FLOOR, "pressure floor"),
                                    (vlct.VLCT_STATUS_DENSITY_FLOOR, "density floor"),
                                    (vlct.VLCT_STATUS_NONFINITE, "non-finite state")) if bits & b]
            raise FloatingPointError("%s: %s (status %d)" % (where, ", ".join(names), bits))

    def ws_adj(self):
        if self._ws_adj is None:
            torch = _torch()
            self._ws_adj = torch.empty(self.ws_adj_bytes, dtype=torch.uint8, device=self.device)
        return self._ws_adj

    def ws_adj_taped(self):
        if self._ws_adj_taped is None:
            torch = _torch()
            self._ws_adj_taped = torch.empty(self.ws_adj_taped_bytes, dtype=torch.uint8,
                                             device=self.device)
        return self._ws_adj_taped

    def new_tape(self):
        torch = _torch()
        return torch.empty(self.tape_bytes, dtype=torch.uint8, device=self.device)

    def empty_state(self) -> Fields:
        torch = _torch()
        return tuple(torch.empty(self.grid.field_shape(f), dtype=torch.float64, device=self.device)
                     for f in FIELDS)

    def _check(self, fields: Sequence) -> Fields:
        torch = _torch()
        out = []
        for f, t in zip(FIELDS, fields):
            if tuple(t.shape) != tuple(self.grid.field_shape(f)):
                raise ValueError("field %s has shape %s, expected %s"
                                 % (f, tuple(t.shape), self.grid.field_shape(f)))
            out.append(t.detach().to(device=self.device, dtype=torch.float64).contiguous())
        return tuple(out)

    @staticmethod
    def c_state(fields: Sequence) -> vlct.vlct_state:
        return vlct.make_state([t.data_ptr() for t in fields])

    def cfl_dt(self, fields: Sequence):
        torch = _torch()
        fields = self._check(fields)
        dt = torch.empty(1, dtype=torch.float64, device=self.device)
        rc = vlct.vlct_cfl_dt(self.cg, self.c_state(fields), dt.data_ptr(), self.ws_step.data_ptr(),
                              self.ws_step_bytes, self._stream())
        if rc:
            raise vlct.VlctError(rc, "vlct_cfl_dt")
        return dt

    def step(self, fields: Sequence, dt, next_dt=None) -> Fields:
        """One step of size dt (a 1-element device tensor) into new arrays;
        next_dt (optional 1-element device tensor) receives the CFL step."""
        fields = self._check(fields)
        out = self.empty_state()
        rc = vlct.vlct_step(self.cg, self.c_state(fields), self.c_state(out), dt.data_ptr(),
                            next_dt.data_ptr() if next_dt is not None else 0,
                            self.status.data_ptr(), self.ws_step.data_ptr(), self.ws_step_bytes,
                            self._stream())
        if rc:
            raise vlct.VlctError(rc, "vlct_step")
        return out

    def step_taped(self, fields: Sequence, dt, tape, next_dt=None) -> Fields:
        """step() that also writes the step's tape (see vlct_step_taped)."""
        fields = self._check(fields)
        out = self.empty_state()
        rc = vlct.vlct_step_taped(self.cg, self.c_state(fields), self.c_state(out), dt.data_ptr(),
                                  next_dt.data_ptr() if next_dt is not None else 0,
                                  self.status.data_ptr(), self.ws_step.data_ptr(),
                                  self.ws_step_bytes, tape.data_ptr(), self.tape_bytes,
                                  self._stream())
        if rc:
            raise vlct.VlctError(rc, "vlct_step_taped")
        return out

    def adjoint_taped(self, fields: Sequence, lam_out: Sequence, dt, tape) -> Fields:
        """adjoint() of a step whose tape step_taped() wrote."""
        fields = self._check(fields)
        lam_out = self._check(lam_out)
        lam_in = self.empty_state()
        ws = self.ws_adj_taped()
        rc = vlct.vlct_step_adjoint_taped(self.cg, self.c_state(fields), self.c_state(lam_out),
                                          self.c_state(lam_in), dt.data_ptr(), tape.data_ptr(),
                                          self.tape_bytes, ws.data_ptr(), self.ws_adj_taped_bytes,
                                          self._stream())
        if rc:
            raise vlct.VlctError(rc, "vlct_step_adjoint_taped")
        return lam_in

    def adjoint(self, fields: Sequence, lam_out: Sequence, dt) -> Fields:
        """lam_in = (d step(fields) / d fields)^T lam_out into new arrays."""
        fields = self._check(fields)
        lam_out = self._check(lam_out)
        lam_in = self.empty_state()
        ws = self.ws_adj()
        rc = vlct.vlct_step_adjoint(self.cg, self.c_state(fields), self.c_state(lam_out),
                                    self.c_state(lam_in), dt.data_ptr(), ws.data_ptr(),
                                    self.ws_adj_bytes, self._stream())
        if rc:
            raise vlct.VlctError(rc, "vlct_step_adjoint")
        return lam_in

    def curl(self, ax, ay, az):
        torch = _torch()
        a = [t.detach().to(device=self.device, dtype=torch.float64).contiguous() for t in (ax, ay, az)]
        for t in a:
            if tuple(t.shape) != tuple(self.grid.field_shape("rho")):
                raise ValueError("vector potential components have the cell shape")
        b = [torch.empty(self.grid.field_shape(f), dtype=torch.float64, device=self.device)
             for f in ("bx", "by", "bz")]
        rc = vlct.vlct_curl_potential(self.cg, *[t.data_ptr() for t in a],
                                      *[t.data_ptr() for t in b], self._stream())
        if rc:
            raise vlct.VlctError(rc, "vlct_curl_potential")
        return tuple(b)

    def curl_adjoint(self, lbx, lby, lbz):
        torch = _torch()
        lb = [t.detach().to(device=self.device, dtype=torch.float64).contiguous()
              for t in (lbx, lby, lbz)]
        la = [torch.empty(self.grid.field_shape("rho"), dtype=torch.float64, device=self.device)
              for _ in range(3)]
        rc = vlct.vlct_curl_potential_adjoint(self.cg, *[t.data_ptr() for t in lb],
                                              *[t.data_ptr() for t in la], self._stream())
        if rc:
            raise vlct.VlctError(rc, "vlct_curl_potential_adjoint")
        return tuple(la)


def _grads_or_zeros(grads, like):
    torch = _torch()
    return tuple(g if g is not None else torch.zeros_like(t) for g, t in zip(grads, like))


def _make_functions():
    torch = _torch()

    class StepFn(torch.autograd.Function):
        """One step of fixed size dt; backward is the step's adjoint."""

        @staticmethod
        def forward(ctx, sim, dt, *fields):
            out = sim.step(fields, dt)
            ctx.sim, ctx.dt = sim, dt
            ctx.save_for_backward(*sim._check(fields))
            return out

        @staticmethod
        def backward(ctx, *grads):
            fields = ctx.saved_tensors
            lam = ctx.sim.adjoint(fields, _grads_or_zeros(grads, fields), ctx.dt)
            return (None, None) + tuple(lam)

    class RolloutFn(torch.autograd.Function):
        """len(dts) steps with checkpoints every `segment` steps; dts are
        1-element device tensors (filled in by the forward pass when
        `record` is set: CFL chain starting from the input state)."""

        @staticmethod
        def forward(ctx, sim, dts, segment, record, taped, *fields):
            cur = sim._check(fields)
            nsteps = len(dts)
            sim.status.zero_()
            if record:
                dts[0].copy_(sim.cfl_dt(cur))
            ckpts = [cur]
            for i in range(nsteps):
                nxt = dts[i + 1] if (record and i + 1 < nsteps) else None
                cur = sim.step(cur, dts[i], nxt)
                if (i + 1) % segment == 0 and i + 1 < nsteps:
                    ckpts.append(cur)
            ctx.sim, ctx.dts, ctx.segment, ctx.nck = sim, list(dts), segment, len(ckpts)
            ctx.taped = taped
            ctx.save_for_backward(*[t for c in ckpts for t in c])
            sim.raise_on_status("rollout forward pass")
            return cur

        @staticmethod
        def backward(ctx, *grads):
            sim, dts, seg = ctx.sim, ctx.dts, ctx.segment
            flat = ctx.saved_tensors
            ckpts = [tuple(flat[8 * c:8 * c + 8]) for c in range(ctx.nck)]
            lam = _grads_or_zeros(grads, ckpts[0])
            nsteps = len(dts)
            sim.status.zero_()
            for s in reversed(range(len(ckpts))):
                start, stop = s * seg, min((s + 1) * seg, nsteps)
                states = [ckpts[s]]
                if ctx.taped:
                    tapes = []
                    for i in range(start, stop):
                        tapes.append(sim.new_tape())
                        nxt = sim.step_taped(states[-1], dts[i], tapes[-1])
                        if i + 1 < stop:
                            states.append(nxt)
                    for i in reversed(range(start, stop)):
                        lam = sim.adjoint_taped(states[i - start], lam, dts[i], tapes[i - start])
                    del tapes
                else:
                    for i in range(start, stop - 1):
                        states.append(sim.step(states[-1], dts[i]))
                    for i in reversed(range(start, stop)):
                        lam = sim.adjoint(states[i - start], lam, dts[i])
                del states
            sim.raise_on_status("rollout backward pass (recomputed segments)")
            return (None, None, None, None, None) + tuple(lam)

    class CurlFn(torch.autograd.Function):
        """Face fields of an edge-centred vector potential, B = curl_h A."""

        @staticmethod
        def forward(ctx, sim, ax, ay, az):
            ctx.sim = sim
            return sim.curl(ax, ay, az)

        @staticmethod
        def backward(ctx, gbx, gby, gbz):
            torch = _torch()
            g = ctx.sim.grid
            lb = [x if x is not None else torch.zeros(g.field_shape(f), dtype=torch.float64,
                                                      device=ctx.sim.device)
                  for x, f in zip((gbx, gby, gbz), ("bx", "by", "bz"))]
            return (None,) + ctx.sim.curl_adjoint(*lb)

    return StepFn, RolloutFn, CurlFn


_FUNCS = None


def _funcs():
    global _FUNCS
    if _FUNCS is None:
        _FUNCS = _make_functions()
    return _FUNCS


def step(sim: Simulator, fields: Sequence, dt) -> Fields:
    """Differentiable single step of size dt (1-element device tensor)."""
    return _funcs()[0].apply(sim, dt, *fields)


def rollout(sim: Simulator, fields: Sequence, nsteps: int = None, dts: Optional[List] = None,
            segment: Optional[int] = None, taped: bool = True):
    """Differentiable rollout with sqrt(N) checkpointing.  Either `dts` (list
    of 1-element device tensors) or `nsteps` (CFL chain recorded by the
    forward pass).  Returns (fields, dts); the backward pass reuses the dts.
    taped=False recomputes each step's fluxes inside its adjoint instead of
    keeping a tape per step of the segment being reversed."""
    torch = _torch()
    record = dts is None
    if record:
        if not nsteps or nsteps < 1:
            raise ValueError("give nsteps >= 1 or a list of step sizes")
        dts = [torch.zeros(1, dtype=torch.float64, device=sim.device) for _ in range(nsteps)]
    n = len(dts)
    seg = segment or max(1, int(math.ceil(math.sqrt(n))))
    out = _funcs()[1].apply(sim, dts, seg, record, bool(taped), *fields)
    return out, dts


def curl(sim: Simulator, ax, ay, az):
    """Differentiable B = curl_h A (face fields with the periodic duplicates)."""
    return _funcs()[2].apply(sim, ax, ay, az)
