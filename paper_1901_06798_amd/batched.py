"""Many patches on one GPU in one persistent launch per (coarse) step.

All patches live in one memory pool per state buffer (the paper's memory pool,
Sec. 4: one large allocation, sub-allocated per patch): three planes, each the
concatenation of every patch's ghost-framed plane.  A patch of level l takes
tref = r^(l-1) substeps per coarse step (Sec. 3: dt refined with dx).  The
step is swe_batched_step followed by swe_cfl_reduce (dt per group on the
device), so a sequence of steps can be captured into a HIP graph and replayed
without host work.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib as L
from .solver import _round_up
from .workloads import Problem


class BatchedSolver:
    def __init__(self, problems, params: L.swe_params | None = None, trefs=None, groups=None,
                 sched: L.swe_schedule | None = None, device: str = "cuda:0",
                 upload: bool = True):
        if not torch.cuda.is_available():
            raise L.SweError("BatchedSolver needs a GPU (torch.cuda is not available)")
        L.lib()
        self.p = params or L.params()
        self.dev_path = self.p.precision != L.F64
        self.dev = torch.device(device)
        self.problems = list(problems)
        n = len(self.problems)
        self.n = n
        self.trefs = list(trefs) if trefs is not None else [1] * n
        self.groups = list(groups) if groups is not None else [0] * n
        self.ngroups = max(self.groups) + 1 if n else 1
        self.sched = sched or L.schedule()
        self.dtype = torch.float32 if self.dev_path else torch.float64
        # pool layout: patch k's plane starts at off[k] within every plane
        offs, total = [], 0
        self.layout = []
        for pb in self.problems:
            pitch = _round_up(pb.mx + 4, 16)
            size = _round_up(pitch * (pb.my + 4), 64)
            offs.append(total)
            self.layout.append((pitch, size))
            total += size
        self.plane = max(total, 64)
        self.patches = []
        for k, pb in enumerate(self.problems):
            pitch, _ = self.layout[k]
            lev = int(pb.meta.get("level", 1)) if pb.meta else 1
            self.patches.append(L.patch(pb.mx, pb.my, pitch, pb.dx, pb.dy, off=offs[k],
                                        plane_stride=self.plane, group=self.groups[k],
                                        tref=self.trefs[k], level=lev, bc=pb.bc))
        self.offs = offs
        self.pools = [torch.zeros(3 * self.plane, dtype=self.dtype, device=self.dev)
                      for _ in range(2)]
        self.work = (torch.zeros(3 * self.plane, dtype=self.dtype, device=self.dev)
                     if max(self.trefs) > 1 else None)
        self.b = torch.zeros(self.plane, dtype=self.dtype, device=self.dev)
        self.cur = 0
        from .solver import patch_table
        self.table = patch_table(self.patches).to(self.dev)
        self.replan(self.sched)
        self.dt = torch.zeros(self.ngroups, dtype=torch.float64, device=self.dev)
        self.smax = torch.zeros(2 * max(n, 1), dtype=torch.float64, device=self.dev)
        self.status = torch.zeros(2, dtype=torch.int32, device=self.dev)
        self.group_flags = torch.zeros(self.ngroups, dtype=torch.int32, device=self.dev)
        self.retake = torch.zeros(self.ngroups, dtype=torch.int32, device=self.dev)
        self.queue = torch.zeros(2, dtype=torch.int32, device=self.dev)
        self.max_mx = max(pb.mx for pb in self.problems)
        self.max_my = max(pb.my for pb in self.problems)
        if upload:  # else the caller writes the pool and the bed itself
            self.upload()
        self.graph = None

    def replan(self, sched: L.swe_schedule) -> None:
        self.sched = sched
        plan = L.swe_batched_plan(self.patches, sched)
        self.nitems, self.ntasks, self.nplain, self.nsub = (plan.nitems, plan.ntasks,
                                                            plan.nplain, plan.nsub)
        self.items, self.tasks = plan.device(self.dev)
        self.graph = None

    @property
    def stream(self) -> int:
        return torch.cuda.current_stream(self.dev).cuda_stream

    def _view(self, flat: torch.Tensor, k: int, nplanes: int):
        pitch, size = self.layout[k]
        pb = self.problems[k]
        rows = pb.my + 4
        v = flat.view(nplanes, self.plane)[:, self.offs[k]: self.offs[k] + pitch * rows]
        return v.reshape(nplanes, rows, pitch)

    def upload(self) -> None:
        """Every patch's initial state from its FP64 arrays: staged in FP64 and
        converted into the pool's precision by swe_state_import."""
        host = torch.zeros(3 * self.plane, dtype=torch.float64)
        hb = torch.zeros(self.plane, dtype=torch.float64)
        for k, pb in enumerate(self.problems):
            Q = self._view(host, k, 3)
            B = self._view(hb, k, 1)[0]
            inner = (slice(2, pb.my + 2), slice(2, pb.mx + 2))
            for c, arr in enumerate((pb.h, pb.hu, pb.hv)):
                Q[c][inner] = torch.from_numpy(np.ascontiguousarray(arr, dtype=np.float64))
            B[inner] = torch.from_numpy(np.ascontiguousarray(pb.b, dtype=np.float64))
        src, src_b = host.to(self.dev), hb.to(self.dev)
        self.pools[self.cur].zero_()
        self.b.zero_()
        L.swe_state_import(self.p, self.table.data_ptr(), self.n, self.max_mx, self.max_my,
                           src.data_ptr(), src_b.data_ptr(), self.pools[self.cur].data_ptr(),
                           self.b.data_ptr(), self.stream)
        L.swe_ghost_fill(self.p, self.table.data_ptr(), self.n, self.max_mx, self.max_my,
                         self.pools[self.cur].data_ptr(), self.b.data_ptr(), 1, self.stream)
        torch.cuda.current_stream(self.dev).synchronize()  # src, src_b are freed below
        self.status.zero_()
        self.smax.zero_()

    def initial_dt(self) -> None:
        self.smax.zero_()
        L.swe_speed_scan(self.p, self.table.data_ptr(), self.n, self.max_mx, self.max_my,
                         self.pools[self.cur].data_ptr(), self.b.data_ptr(), self.smax.data_ptr(),
                         self.stream)
        L.swe_cfl_reduce(self.p, self.table.data_ptr(), self.n, self.ngroups, self.smax.data_ptr(),
                         self.dt.data_ptr(), self.status.data_ptr(), self.group_flags.data_ptr(), 1,
                         self.stream)

    def enqueue_step(self, cfl: bool = True, dt_ptr: int | None = None,
                     retake: bool = True) -> None:
        """One coarse step of every patch: pools[cur] -> pools[1 - cur].  With
        cfl the CFL reduction writes each group's next dt; with retake as
        well, the groups whose step went above cfl_max are redone once on the
        device with their reduced dt."""
        args = (self.table.data_ptr(), self.items.data_ptr(), self.nitems,
                self.tasks.data_ptr(),
                self.tasks.data_ptr() + L.SWE_TASK_BYTES * (self.ntasks - self.nplain),
                self.nplain, self.nsub, self.pools[self.cur].data_ptr(),
                self.pools[1 - self.cur].data_ptr(),
                self.work.data_ptr() if self.work is not None else 0, 3 * self.plane,
                self.b.data_ptr())
        L.swe_batched_step(self.p, *args, dt_ptr if dt_ptr is not None else self.dt.data_ptr(),
                           self.smax.data_ptr(), self.status.data_ptr(), self.queue.data_ptr(),
                           self.sched, self.stream)
        if cfl:
            rt = self.retake.data_ptr() if retake else 0
            L.swe_cfl_reduce(self.p, self.table.data_ptr(), self.n, self.ngroups,
                             self.smax.data_ptr(), self.dt.data_ptr(), self.status.data_ptr(),
                             self.group_flags.data_ptr(), 0, self.stream, retake=rt)
            if retake:
                L.swe_batched_retake(self.p, *args, self.dt.data_ptr(), self.smax.data_ptr(),
                                     self.status.data_ptr(), self.queue.data_ptr(), self.sched,
                                     rt, self.ngroups, self.stream)
                L.swe_cfl_reduce(self.p, self.table.data_ptr(), self.n, self.ngroups,
                                 self.smax.data_ptr(), self.dt.data_ptr(),
                                 self.status.data_ptr(), self.group_flags.data_ptr(), 0,
                                 self.stream)
        self.cur ^= 1

    def run(self, nsteps: int, record_dt: bool = False):
        dts = []
        for _ in range(nsteps):
            if record_dt:
                dts.append(self.dt.clone())
            self.enqueue_step()
        if record_dt:
            return torch.stack(dts).cpu().numpy()
        return None

    def capture(self, nsteps: int) -> None:
        """Capture nsteps (even) coarse steps into a HIP graph."""
        if nsteps % 2:
            raise ValueError("capture an even number of steps so the buffers return")
        s = torch.cuda.Stream(self.dev)
        s.wait_stream(torch.cuda.current_stream(self.dev))
        g = torch.cuda.CUDAGraph()
        with torch.cuda.stream(s):
            # warm the allocator and the launch path outside the capture
            torch.cuda.synchronize(self.dev)
            with torch.cuda.graph(g, stream=s):
                for _ in range(nsteps):
                    self.enqueue_step()
        torch.cuda.current_stream(self.dev).wait_stream(s)
        self.graph = g
        self.graph_steps = nsteps

    def replay(self) -> None:
        self.graph.replay()

    # -- results -------------------------------------------------------------
    def state(self, k: int):
        pb = self.problems[k]
        Q = self._view(self.pools[self.cur], k, 3).cpu().numpy().astype(np.float64)
        inner = (slice(2, pb.my + 2), slice(2, pb.mx + 2))
        h = Q[0][inner].copy()
        if self.dev_path:
            B = self._view(self.b, k, 1)[0].cpu().numpy().astype(np.float64)
            h = (h + self.p.sea_level) - B[inner]
        return h, Q[1][inner].copy(), Q[2][inner].copy()

    def surface(self, k: int):
        pb = self.problems[k]
        Q = self._view(self.pools[self.cur], k, 3).cpu().numpy().astype(np.float64)
        inner = (slice(2, pb.my + 2), slice(2, pb.mx + 2))
        if self.dev_path:
            return Q[0][inner] + self.p.sea_level
        B = self._view(self.b, k, 1)[0].cpu().numpy()
        return Q[0][inner] + B[inner]

    def flags(self):
        st = self.status.cpu().numpy()
        return int(st[0]), int(st[1])

    def cells(self) -> int:
        return sum(pb.mx * pb.my * t for pb, t in zip(self.problems, self.trefs))
