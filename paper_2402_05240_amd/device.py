"""Device-resident state for the VL+CT library: torch tensors provide HBM and
the stream, every computation runs in libvlct.so through the C ABI."""
from __future__ import annotations

from typing import Dict

import numpy as np

from . import vlct
from .inputs import FIELDS, Grid


def _torch():
    import torch
    return torch


class DeviceState:
    """Eight FP64 device arrays in the layout of include/vlct.h."""

    def __init__(self, grid: Grid, device: str = "cuda:0"):
        torch = _torch()
        self.grid = grid
        self.t = {f: torch.empty(grid.field_shape(f), dtype=torch.float64, device=device)
                  for f in FIELDS}

    def ptrs(self):
        return [self.t[f].data_ptr() for f in FIELDS]

    def c_state(self) -> vlct.vlct_state:
        return vlct.make_state(self.ptrs())

    def upload(self, s: Dict[str, np.ndarray]) -> "DeviceState":
        torch = _torch()
        for f in FIELDS:
            self.t[f].copy_(torch.from_numpy(np.ascontiguousarray(s[f], dtype=np.float64)))
        return self

    def download(self) -> Dict[str, np.ndarray]:
        return {f: self.t[f].cpu().numpy() for f in FIELDS}


class Stepper:
    """Owns the workspace and the device dt words; steps ping-pong between two
    states (or in place) on torch's current stream."""

    def __init__(self, grid: Grid, device: str = "cuda:0", inplace: bool = False):
        torch = _torch()
        self.grid = grid
        self.device = device
        self.cg = vlct.make_grid(grid)
        self.ws_bytes = vlct.vlct_workspace_bytes(self.cg)
        if self.ws_bytes == 0:
            raise ValueError("invalid grid descriptor")
        self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device=device)
        self.cur = DeviceState(grid, device)
        self.nxt = self.cur if inplace else DeviceState(grid, device)
        self.dt = torch.zeros(1, dtype=torch.float64, device=device)
        self.next_dt = torch.zeros(1, dtype=torch.float64, device=device)
        self.status = torch.zeros(1, dtype=torch.int32, device=device)

    def stream(self) -> int:
        return _torch().cuda.current_stream().cuda_stream

    def upload(self, s):
        self.cur.upload(s)
        return self

    def download(self):
        return self.cur.download()

    def compute_dt(self) -> None:
        rc = vlct.vlct_cfl_dt(self.cg, self.cur.c_state(), self.dt.data_ptr(), self.ws.data_ptr(),
                              self.ws_bytes, self.stream())
        if rc:
            raise vlct.VlctError(rc, "vlct_cfl_dt")

    def set_dt(self, dt: float) -> None:
        self.dt.fill_(float(dt))

    def step(self) -> None:
        """One step of size self.dt; afterwards self.dt holds the next CFL step."""
        rc = vlct.vlct_step(self.cg, self.cur.c_state(), self.nxt.c_state(), self.dt.data_ptr(),
                            self.next_dt.data_ptr(), self.status.data_ptr(), self.ws.data_ptr(),
                            self.ws_bytes, self.stream())
        if rc:
            raise vlct.VlctError(rc, "vlct_step")
        self.cur, self.nxt = self.nxt, self.cur
        self.dt, self.next_dt = self.next_dt, self.dt

    def step_observed(self, cb) -> None:
        """step() through vlct_step_observed: cb(kernel, phase, stream) runs on
        this thread around each kernel launch of the step (profiling)."""
        rc = vlct.vlct_step_observed(self.cg, self.cur.c_state(), self.nxt.c_state(),
                                     self.dt.data_ptr(), self.next_dt.data_ptr(),
                                     self.status.data_ptr(), self.ws.data_ptr(), self.ws_bytes,
                                     self.stream(), cb)
        if rc:
            raise vlct.VlctError(rc, "vlct_step_observed")
        self.cur, self.nxt = self.nxt, self.cur
        self.dt, self.next_dt = self.next_dt, self.dt

    def status_bits(self) -> int:
        return int(self.status.item())


class BatchStepper:
    """Independent instances advanced together by vlct_step_batch (one launch
    per kernel for all of them); per-instance dt, next dt and status live in
    device arrays of len(grids) elements."""

    def __init__(self, grids, device: str = "cuda:0", inplace: bool = False, plan=None):
        torch = _torch()
        self.plan = list(plan) if plan is not None else None
        self.grids = list(grids)
        n = len(self.grids)
        self.device = device
        self.cgs = [vlct.make_grid(g) for g in self.grids]
        self.ws_bytes = vlct.vlct_batch_workspace_bytes(self.cgs)
        if self.ws_bytes == 0:
            raise ValueError("invalid grid descriptors")
        self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device=device)
        self.cur = [DeviceState(g, device) for g in self.grids]
        self.nxt = self.cur if inplace else [DeviceState(g, device) for g in self.grids]
        self.dt = torch.zeros(n, dtype=torch.float64, device=device)
        self.next_dt = torch.zeros(n, dtype=torch.float64, device=device)
        self.status = torch.zeros(n, dtype=torch.int32, device=device)

    def stream(self) -> int:
        return _torch().cuda.current_stream().cuda_stream

    def upload(self, states):
        for d, s in zip(self.cur, states):
            d.upload(s)
        return self

    def download(self):
        return [d.download() for d in self.cur]

    def set_dt(self, dts) -> None:
        torch = _torch()
        self.dt.copy_(torch.tensor([float(x) for x in dts], dtype=torch.float64))

    def compute_dt(self) -> None:
        """CFL step of every instance (one vlct_cfl_dt each; the batch
        workspace is larger than any single instance needs)."""
        for i, (cg, d) in enumerate(zip(self.cgs, self.cur)):
            rc = vlct.vlct_cfl_dt(cg, d.c_state(), self.dt.data_ptr() + 8 * i,
                                  self.ws.data_ptr(), self.ws_bytes, self.stream())
            if rc:
                raise vlct.VlctError(rc, "vlct_cfl_dt")

    def step(self) -> None:
        """One step of every instance; afterwards self.dt holds the next CFL steps."""
        rc = vlct.vlct_step_batch_plan(self.cgs, [d.c_state() for d in self.cur],
                                       [d.c_state() for d in self.nxt], self.dt.data_ptr(),
                                       self.next_dt.data_ptr(), self.status.data_ptr(),
                                       self.plan, self.ws.data_ptr(), self.ws_bytes, self.stream())
        if rc:
            raise vlct.VlctError(rc, "vlct_step_batch_plan")
        self.cur, self.nxt = self.nxt, self.cur
        self.dt, self.next_dt = self.next_dt, self.dt

    def run_until(self, t_end, check_every: int = 8, max_steps: int = 100000):
        """Advance every instance in place to its own end time t_end[i]
        (vlct_step_batch_until: the last step of each is clipped to land on
        it, finished instances drop out of the kernels on the device).  Every
        `check_every` steps the host reads the times and launches only the
        instances still running from then on (their dt, next dt, status and
        time gathered into compact device arrays), so a long-running few no
        longer carry the empty blocks of the rest.  Returns the number of
        batched steps."""
        torch = _torch()
        if self.nxt is not self.cur:
            raise ValueError("run_until steps in place")
        n = len(self.grids)
        self.t = torch.zeros(n, dtype=torch.float64, device=self.device)
        tend = torch.tensor([float(x) for x in t_end], dtype=torch.float64, device=self.device)
        active = list(range(n))
        steps = 0
        while active and steps < max_steps:
            idx = torch.tensor(active, dtype=torch.long, device=self.device)
            t_a, te_a = self.t[idx].contiguous(), tend[idx].contiguous()
            dt_a, st_a = self.dt[idx].contiguous(), self.status[idx].contiguous()
            nd_a = torch.empty_like(dt_a)
            grids = [self.cgs[i] for i in active]
            states = [self.cur[i].c_state() for i in active]
            plan = [self.plan[i] for i in active] if self.plan is not None else None
            for _ in range(check_every):
                rc = vlct.vlct_step_batch_until(grids, states, dt_a.data_ptr(), nd_a.data_ptr(),
                                                st_a.data_ptr(), t_a.data_ptr(), te_a.data_ptr(),
                                                plan, self.ws.data_ptr(), self.ws_bytes,
                                                self.stream())
                if rc:
                    raise vlct.VlctError(rc, "vlct_step_batch_until")
                # a finished instance keeps its dt; a running one takes its next CFL step
                dt_a.copy_(torch.where(t_a < te_a, nd_a, dt_a))
                steps += 1
            self.t[idx] = t_a
            self.dt[idx] = dt_a
            self.status[idx] = st_a
            running = (t_a < te_a).cpu().tolist()
            active = [i for i, r in zip(active, running) if r]
        return steps

    def tune(self, reps: int = 3):
        """Per-instance tiles from the library's autotuner (vlct_batch_tune),
        timed on the current states with the current dt; needs out-of-place
        stepping (the trial steps overwrite the other buffer)."""
        if self.nxt is self.cur:
            raise ValueError("tuning needs out-of-place stepping")
        rc, plan = vlct.vlct_batch_tune(self.cgs, [d.c_state() for d in self.cur],
                                        [d.c_state() for d in self.nxt], self.dt.data_ptr(),
                                        self.ws.data_ptr(), self.ws_bytes, self.stream(), reps)
        if rc:
            raise vlct.VlctError(rc, "vlct_batch_tune")
        self.plan = plan
        return plan

    def status_bits(self):
        return [int(x) for x in self.status.cpu()]


class Adjoint:
    """Reverse derivative of one step (vlct_step_adjoint): for a state at the
    start of a step of fixed size dt, maps the cotangent of the step's output
    to the cotangent of its input.  Owns the workspace and three states."""

    def __init__(self, grid: Grid, device: str = "cuda:0"):
        torch = _torch()
        self.grid = grid
        self.cg = vlct.make_grid(grid)
        self.ws_bytes = vlct.vlct_adjoint_workspace_bytes(self.cg)
        if self.ws_bytes == 0:
            raise ValueError("invalid grid descriptor")
        self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device=device)
        self.state = DeviceState(grid, device)
        self.lam_out = DeviceState(grid, device)
        self.lam_in = DeviceState(grid, device)
        self.dt = torch.zeros(1, dtype=torch.float64, device=device)

    def stream(self) -> int:
        return _torch().cuda.current_stream().cuda_stream

    def run(self) -> None:
        """lam_in = (d step / d state)^T lam_out on the device-resident arrays."""
        rc = vlct.vlct_step_adjoint(self.cg, self.state.c_state(), self.lam_out.c_state(),
                                    self.lam_in.c_state(), self.dt.data_ptr(),
                                    self.ws.data_ptr(), self.ws_bytes, self.stream())
        if rc:
            raise vlct.VlctError(rc, "vlct_step_adjoint")

    def vjp(self, s: Dict[str, np.ndarray], lam_out: Dict[str, np.ndarray],
            dt: float) -> Dict[str, np.ndarray]:
        """Host round trip: upload the state and lam_out, run, download lam_in."""
        self.state.upload(s)
        self.lam_out.upload(lam_out)
        self.dt.fill_(float(dt))
        self.run()
        return self.lam_in.download()
