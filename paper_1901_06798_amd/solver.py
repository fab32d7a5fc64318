"""Device-resident single-patch solver on top of the C ABI.

PyTorch provides the device memory and the stream; every step of the method
runs in the HIP library (libswe.so).  The state is double-buffered SoA planes
(h, hu, hv) in FP64, or (eta', hu, hv) in FP32 with eta' = h + b - sea_level
on the surface-deviation path, plus the bathymetry plane; rows are padded to
128-byte multiples.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib as L
from .workloads import Problem


def _round_up(x: int, m: int) -> int:
    return (x + m - 1) // m * m


def patch_table(patches) -> torch.Tensor:
    """Bytes of a swe_patch array as a uint8 CPU tensor."""
    n = len(patches)
    arr = (L.swe_patch * n)(*patches)
    return torch.frombuffer(bytearray(bytes(arr)), dtype=torch.uint8)


class PatchSolver:
    """One patch on one GPU with the CFL rule of Sec. 2 (dt from the previous
    step's speeds, a step above cfl_max is retaken with the reduced dt)."""

    def __init__(self, pb: Problem, params: L.swe_params | None = None, device: str = "cuda:0",
                 ordered: bool = True, order_every: int = 4, launch: L.swe_launch | None = None):
        if not torch.cuda.is_available():
            raise L.SweError("PatchSolver needs a GPU (torch.cuda is not available)")
        L.lib()
        self.pb = pb
        self.p = params or L.params()
        self.dev_path = self.p.precision != L.F64
        self.dev = torch.device(device)
        self.mx, self.my = pb.mx, pb.my
        self.pitch = _round_up(self.mx + 4, 16)
        self.rows = self.my + 4
        self.ps = _round_up(self.pitch * self.rows, 64)
        f64 = torch.float64
        self.dtype = torch.float32 if self.dev_path else f64
        self.q = [torch.zeros(3 * self.ps, dtype=self.dtype, device=self.dev) for _ in range(2)]
        self.b = torch.zeros(self.ps, dtype=self.dtype, device=self.dev)
        self.cur = 0
        self.pt = L.patch(self.mx, self.my, self.pitch, pb.dx, pb.dy, off=0, plane_stride=self.ps,
                          bc=pb.bc)
        self.pt_dev = patch_table([self.pt]).to(self.dev)
        self.dt = torch.zeros(1, dtype=f64, device=self.dev)
        self.smax = torch.zeros(2, dtype=f64, device=self.dev)
        self.status = torch.zeros(2, dtype=torch.int32, device=self.dev)
        self.retake = torch.zeros(1, dtype=torch.int32, device=self.dev)
        # finished-wave counter of the launches that end with the CFL rule
        self.counter = torch.zeros(3, dtype=torch.int32, device=self.dev)
        self.fused = True  # the step and the CFL rule in one launch
        self.metric_ptr = 0
        # launch order of the step's tasks, heaviest first from the last step
        # (re-sorted after the first step, then every order_every steps: the
        # work of a task changes slowly as the waves travel)
        # (launch: the step's launch shape, None = the library's defaults; a
        # schedule buffer that is never sorted keeps the tasks in index order)
        self.launch = launch
        self.ordered = ordered
        self.sched = (torch.zeros(L.swe_workspace_bytes(self.pt, launch) // 4, dtype=torch.int32,
                                  device=self.dev) if ordered or launch is not None else None)
        self.order_every = max(1, int(order_every))
        self.steps_launched = 0
        self.upload(pb)

    # -- layout helpers ------------------------------------------------------
    def planes(self, k: int | None = None) -> torch.Tensor:
        k = self.cur if k is None else k
        return self.q[k].view(3, self.ps)[:, : self.pitch * self.rows].view(3, self.rows, self.pitch)

    def bplane(self) -> torch.Tensor:
        return self.b[: self.pitch * self.rows].view(self.rows, self.pitch)

    @property
    def stream(self) -> int:
        return torch.cuda.current_stream(self.dev).cuda_stream

    def upload(self, pb: Problem) -> None:
        """Initial state from FP64 arrays, converted on the device into the
        planes' precision (swe_state_import), then the ghost frame."""
        self.planes().zero_()
        self.b.zero_()
        inner = (slice(2, self.my + 2), slice(2, self.mx + 2))
        src = torch.zeros(3, self.rows, self.pitch, dtype=torch.float64)
        src_b = torch.zeros(self.rows, self.pitch, dtype=torch.float64)
        for k, arr in enumerate((pb.h, pb.hu, pb.hv)):
            src[k][inner] = torch.from_numpy(np.ascontiguousarray(arr, dtype=np.float64))
        src_b[inner] = torch.from_numpy(np.ascontiguousarray(pb.b, dtype=np.float64))
        # the FP64 staging planes take the state planes' element layout
        dsrc = torch.zeros(3 * self.ps, dtype=torch.float64, device=self.dev)
        dsrc.view(3, self.ps)[:, : self.pitch * self.rows].copy_(src.view(3, -1))
        dsrc_b = src_b.view(-1).to(self.dev)
        L.swe_state_import(self.p, self.pt_dev.data_ptr(), 1, self.mx, self.my, dsrc.data_ptr(),
                           dsrc_b.data_ptr(), self.q[self.cur].data_ptr(), self.b.data_ptr(),
                           self.stream)
        self.ghost_fill(fill_b=True)
        torch.cuda.current_stream(self.dev).synchronize()  # before the staging planes go
        self.status.zero_()
        self.smax.zero_()

    # -- library calls -------------------------------------------------------
    def ghost_fill(self, fill_b: bool = False) -> None:
        L.swe_ghost_fill(self.p, self.pt_dev.data_ptr(), 1, self.mx, self.my,
                         self.q[self.cur].data_ptr(), self.b.data_ptr(), int(fill_b), self.stream)

    def launch_scan(self) -> None:
        """Speeds of the current state's Riemann problems into smax."""
        L.swe_speed_scan(self.p, self.pt_dev.data_ptr(), 1, self.mx, self.my,
                         self.q[self.cur].data_ptr(), self.b.data_ptr(), self.smax.data_ptr(),
                         self.stream)

    def initial_dt(self) -> None:
        self.smax.zero_()
        self.launch_scan()
        L.swe_cfl_reduce(self.p, self.pt_dev.data_ptr(), 1, 1, self.smax.data_ptr(),
                         self.dt.data_ptr(), self.status.data_ptr(), 0, 1, self.stream)

    def launch_step(self, qi: int, qo: int, dt: int, stream: int | None = None) -> None:
        """The step launch alone: q_out = step(q_in, *dt)."""
        st = self.stream if stream is None else stream
        if self.sched is not None:
            L.swe_patch_step_sched(self.p, self.pt, qi, qo, self.b.data_ptr(), dt,
                                   self.smax.data_ptr(), self.status.data_ptr(),
                                   self.sched.data_ptr(), self.sched.numel(), self.launch, st)
        else:
            L.swe_patch_step(self.p, self.pt, qi, qo, self.b.data_ptr(), dt,
                             self.smax.data_ptr(), self.status.data_ptr(), st)

    def launch_step_cfl(self, qi: int, qo: int, stream: int | None = None) -> None:
        """The step with dt from self.dt, ending with the CFL rule (next dt,
        retake flag) in its last wave."""
        L.swe_patch_step_cfl(self.p, self.pt, qi, qo, self.b.data_ptr(), self.dt.data_ptr(),
                             self.smax.data_ptr(), self.status.data_ptr(),
                             self.retake.data_ptr(), self.counter.data_ptr(), self.metric_ptr,
                             self.sched.data_ptr() if self.sched is not None else 0,
                             self.sched.numel() if self.sched is not None else 0, self.launch,
                             self.stream if stream is None else stream)

    def launch_retake_cfl(self, qi: int, qo: int, stream: int | None = None,
                          last: int = 1) -> None:
        """The gated redo of the step, ending with the CFL rule when it runs
        (last = 0: a redo still above the limit asks for one more)."""
        L.swe_patch_retake_cfl(self.p, self.pt, qi, qo, self.b.data_ptr(), self.dt.data_ptr(),
                               self.smax.data_ptr(), self.status.data_ptr(),
                               self.retake.data_ptr(), self.counter.data_ptr(), self.metric_ptr,
                               last, self.stream if stream is None else stream)

    def launch_retake(self, qi: int, qo: int, retake: int, stream: int | None = None) -> None:
        """The gated redo of the step q_in -> q_out with the reduced dt."""
        L.swe_patch_retake(self.p, self.pt, qi, qo, self.b.data_ptr(), self.dt.data_ptr(),
                           self.smax.data_ptr(), self.status.data_ptr(), retake,
                           self.stream if stream is None else stream)

    def launch_order(self, stream: int | None = None) -> None:
        """Next step's launch order from this step's work (ordered solvers)."""
        if self.ordered:
            L.swe_patch_order(self.pt, self.sched.data_ptr(), self.sched.numel(), self.launch,
                              self.stream if stream is None else stream)

    def after_step(self, stream: int | None = None) -> None:
        """Count a step launch and re-sort the launch order when it is due."""
        self.steps_launched += 1
        if self.steps_launched % self.order_every == 1 or self.order_every == 1:
            self.launch_order(stream)

    def enqueue_step(self, dt_ptr: int | None = None, cfl: bool = True,
                     retake: bool = True) -> None:
        """One step q[cur] -> q[1 - cur]; dt from dt_ptr (device) or self.dt.
        With cfl, the CFL reduction writes the next dt; with retake as well, a
        step above cfl_max is redone on the device with the reduced dt: up to
        twice when the rule is fused into the launches (the default), once
        with the separate reduction launches; a last redo still above the
        limit stands and is flagged CFL_EXCEEDED."""
        qi, qo = self.q[self.cur].data_ptr(), self.q[1 - self.cur].data_ptr()
        if cfl and retake and dt_ptr is None and self.fused:
            self.launch_step_cfl(qi, qo)
            self.after_step()
            # up to two redos, each a gated launch that ends at once unless due
            self.launch_retake_cfl(qi, qo, last=0)
            self.launch_retake_cfl(qi, qo, last=1)
            self.cur ^= 1
            return
        dt = dt_ptr if dt_ptr is not None else self.dt.data_ptr()
        self.launch_step(qi, qo, dt)
        self.after_step()
        if cfl:
            rt = self.retake.data_ptr() if retake else 0
            L.swe_cfl_reduce(self.p, self.pt_dev.data_ptr(), 1, 1, self.smax.data_ptr(),
                             self.dt.data_ptr(), self.status.data_ptr(), 0, 0, self.stream,
                             retake=rt)
            if retake:
                self.launch_retake(qi, qo, rt)
                L.swe_cfl_reduce(self.p, self.pt_dev.data_ptr(), 1, 1, self.smax.data_ptr(),
                                 self.dt.data_ptr(), self.status.data_ptr(), 0, 0, self.stream)
        self.cur ^= 1

    def run(self, nsteps: int, dt0: float | None = None, record_dt: bool = True):
        """Advance nsteps accepted steps with the CFL rule, checking the status
        after every step (a flagged step is retaken with the reduced dt).
        Returns the accepted step sizes."""
        if dt0 is None:
            self.initial_dt()
        else:
            self.dt.fill_(dt0)
        dts = []
        retakes = 0
        s = 0
        while s < nsteps:
            dt_now = self.dt.clone() if record_dt else None
            before = self.status.clone()
            self.enqueue_step(retake=False)
            st = self.status.cpu()
            if int(st[0]) & L.STATUS_CFL_EXCEEDED:
                # discard: the output buffer is dropped and the step retaken with
                # the reduced dt that the CFL reduction just wrote; what the
                # discarded step reported is dropped with it
                self.cur ^= 1
                self.status.copy_(before)
                retakes += 1
                continue
            if record_dt:
                dts.append(float(dt_now.item()))
            s += 1
        self.retakes = retakes
        return np.array(dts)

    def run_forced(self, dts) -> None:
        """Advance with a given dt sequence (no CFL control)."""
        sched = torch.as_tensor(np.asarray(dts, dtype=np.float64), device=self.dev)
        for k in range(len(dts)):
            self.enqueue_step(sched.data_ptr() + 8 * k, cfl=False)
            self.smax.zero_()

    def run_async(self, nsteps: int) -> None:
        """Enqueue nsteps with the CFL rule on the device, without host checks."""
        for _ in range(nsteps):
            self.enqueue_step()

    # -- results -------------------------------------------------------------
    def state(self):
        """Interior (h, hu, hv) as float64 arrays."""
        Q = self.planes().cpu().numpy().astype(np.float64)
        inner = (slice(2, self.my + 2), slice(2, self.mx + 2))
        h = Q[0][inner].copy()
        if self.dev_path:
            b = self.bplane().cpu().numpy().astype(np.float64)[inner]
            h = (h + self.p.sea_level) - b
        return h, Q[1][inner].copy(), Q[2][inner].copy()

    def surface(self):
        """Interior surface elevation h + b (eta' + sea level on the deviation path)."""
        Q = self.planes().cpu().numpy().astype(np.float64)
        inner = (slice(2, self.my + 2), slice(2, self.mx + 2))
        if self.dev_path:
            return Q[0][inner] + self.p.sea_level
        return Q[0][inner] + self.bplane().cpu().numpy()[inner]

    def flags(self):
        st = self.status.cpu().numpy()
        return int(st[0]), int(st[1])

    def mass(self) -> float:
        out = torch.zeros(1, dtype=torch.float64, device=self.dev)
        L.swe_mass(self.p, self.pt_dev.data_ptr(), 1, self.q[self.cur].data_ptr(),
                   self.b.data_ptr(), out.data_ptr(), self.stream)
        return float(out.item())
