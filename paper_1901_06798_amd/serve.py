"""Continuous batching of tsunami scenario solves on one GPU.

Early warning needs fast results (the paper's motivation, Sec. 1).  Requests
(one grid each, of its own size) arrive over time.  The server keeps every
admitted scenario's state resident in HBM, in one pool per state buffer
(first-fit sub-allocation of one large allocation, the paper's memory pool of
Sec. 4), and advances all active scenarios together: each round is R steps of
swe_batched_step + swe_cfl_reduce, every scenario in its own dt group, so a
scenario's result does not depend on who else is in the batch.  Between
rounds it retires finished scenarios and admits queued ones while a slot is
free and their HBM footprint fits the budget.  Latency is arrival to
completion (result on the host).

The host stays one round ahead of the device: all device work (uploads,
rounds, result copies) is ordered on one stream, uploads and result copies go
through pinned staging buffers without blocking, and the host waits only for
the round before the one it just queued.  A retired scenario's pool range and
slot can be handed to a new scenario at once, because the new scenario's
upload is queued after the old scenario's last copy.
"""
from __future__ import annotations

import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np
import torch

from . import _lib as L
from .timeline import markers
from .solver import _round_up, patch_table
from .workloads import Problem


def admit_in_order(queue: list, try_admit, now: float, max_bypass_s: float) -> list:
    """Admission of waiting requests (queue in arrival order; try_admit(sc)
    admits sc if a slot is free and its footprint fits, and says whether it
    did).  Requests are tried oldest first; one that does not fit is passed
    over by later ones that do (small grids fill memory that a large one is
    waiting for), until it has waited longer than max_bypass_s: from then on
    nothing is admitted ahead of it, so no request waits behind newer ones
    for longer than that.  max_bypass_s <= 0: strict arrival order.  Removes
    the admitted requests from queue and returns them."""
    admitted = []
    k = 0
    while k < len(queue):
        sc = queue[k]
        if try_admit(sc):
            admitted.append(queue.pop(k))
            continue
        if max_bypass_s <= 0 or now - sc.arrival > max_bypass_s:
            break
        k += 1
    return admitted


class PoolAllocator:
    """First-fit allocator of element ranges within one pool; 256-byte aligned."""

    def __init__(self, size: int, align: int = 64):
        self.size = size
        self.align = align
        self.free = [(0, size)]  # sorted (start, length)

    def alloc(self, n: int):
        n = _round_up(n, self.align)
        for i, (s, ln) in enumerate(self.free):
            if ln >= n:
                if ln == n:
                    self.free.pop(i)
                else:
                    self.free[i] = (s + n, ln - n)
                return s, n
        return None

    def release(self, start: int, n: int) -> None:
        self.free.append((start, n))
        self.free.sort()
        merged = []
        for s, ln in self.free:
            if merged and merged[-1][0] + merged[-1][1] == s:
                merged[-1] = (merged[-1][0], merged[-1][1] + ln)
            else:
                merged.append((s, ln))
        self.free = merged

    def largest_free(self) -> int:
        return max((ln for _, ln in self.free), default=0)


@dataclass
class Scenario:
    """One request: its grid as host arrays (`problem`) or as seeded parameters
    built on the device at admission (`spec`, a workloads.ScenarioSpec)."""
    rid: int
    arrival: float
    problem: Problem | None
    nsteps: int
    spec: object = None
    slot: int = -1
    off: int = 0
    span: int = 0
    steps_done: int = 0
    admitted: float = 0.0
    finished: float = 0.0
    state: str = "queued"  # queued, active, done, rejected, cancelled
    reason: str = ""
    result: dict = field(default_factory=dict)

    @property
    def grid(self):
        """Geometry (mx, my, dx, dy, bc) of the request."""
        return self.problem if self.problem is not None else self.spec


class PinnedPool:
    """Pinned host buffers, reused once the copies that use them are done."""

    def __init__(self, dtype: torch.dtype):
        self.dtype = dtype
        self.free: list[torch.Tensor] = []

    def get(self, n: int) -> torch.Tensor:
        best = None
        for k, t in enumerate(self.free):
            if t.numel() >= n and (best is None or t.numel() < self.free[best].numel()):
                best = k
        if best is not None:
            return self.free.pop(best)[:n]
        return torch.empty(max(n, 1 << 16), dtype=self.dtype, pin_memory=True)[:n]

    def put(self, t: torch.Tensor) -> None:
        base = t._base if t._base is not None else t
        self.free.append(base)


class ScenarioServer:
    def __init__(self, params: L.swe_params | None = None, hbm_budget: int = 64 << 30,
                 max_slots: int = 64, steps_per_round: int = 50, device: str = "cuda:0",
                 sched: L.swe_schedule | None = None, graphs: bool = False,
                 max_bypass_s: float = 0.0):
        if not torch.cuda.is_available():
            raise L.SweError("ScenarioServer needs a GPU")
        L.lib()
        self.p = params or L.params(precision=L.F32_DEV)
        self.dev = torch.device(device)
        self.dtype = torch.float32 if self.p.precision == L.F32_DEV else torch.float64
        self.esize = 4 if self.p.precision == L.F32_DEV else 8
        self.R = steps_per_round
        self.max_slots = max_slots
        # a request that does not fit may be passed over by later ones for
        # this long (admit_in_order); 0: strict arrival order, which gave the
        # lower p99 on the memory-bound stream (a passed-over large grid then
        # waits for several smaller ones)
        self.max_bypass_s = max_bypass_s
        self.sched = sched or L.schedule(seg=64, waves_per_group=4)
        # one plane of the pool holds every scenario's plane; 7 planes in total
        # (2 x 3 state planes + bathymetry)
        self.plane = _round_up(hbm_budget // (7 * self.esize), 64)
        self.alloc = PoolAllocator(self.plane)
        self.pools = [torch.zeros(3 * self.plane, dtype=self.dtype, device=self.dev)
                      for _ in range(2)]
        self.b = torch.zeros(self.plane, dtype=self.dtype, device=self.dev)
        self.dt = torch.zeros(max_slots, dtype=torch.float64, device=self.dev)
        self.smax = torch.zeros(2 * max_slots, dtype=torch.float64, device=self.dev)
        self.status = torch.zeros(2, dtype=torch.int32, device=self.dev)
        # per scenario slot: (status bits, depth resets) of its own steps
        self.gstatus = torch.zeros(2 * max_slots, dtype=torch.int32, device=self.dev)
        self.group_flags = torch.zeros(max_slots, dtype=torch.int32, device=self.dev)
        self.retake = torch.zeros(max_slots, dtype=torch.int32, device=self.dev)
        # each step's conditions per slot until the CFL rule settles them
        self.pending = torch.zeros(2 * max_slots, dtype=torch.int32, device=self.dev)
        self.queue_ctr = torch.zeros(2, dtype=torch.int32, device=self.dev)
        self.cur = 0
        self.active: list[Scenario] = []
        self.free_slots = list(range(max_slots))
        self.table_dirty = True
        self.host_state = PinnedPool(self.dtype)
        self.host_f64 = PinnedPool(torch.float64)
        self.host_bytes = PinnedPool(torch.uint8)
        self.host_status = PinnedPool(torch.int32)
        self.hold: list = []  # pinned buffers read by copies not yet known to be done
        # rounds captured as HIP graphs, per (state buffer, steps), valid until
        # the active set changes
        self.use_graphs = graphs
        self.graphs: dict = {}
        self.rsmax = None

    @property
    def stream(self) -> int:
        return torch.cuda.current_stream(self.dev).cuda_stream

    def _to_device(self, host: torch.Tensor) -> torch.Tensor:
        """Asynchronous copy of a small CPU tensor through pinned memory."""
        st = self.host_bytes.get(host.numel())
        st.copy_(host)
        self.hold.append((self.host_bytes, st))
        return st.to(self.dev, non_blocking=True)

    # -- footprint and admission ----------------------------------------------
    def footprint_elems(self, pb) -> int:
        pitch = _round_up(pb.mx + 4, 16)
        return _round_up(pitch * (pb.my + 4), 64)

    def footprint_bytes(self, pb) -> int:
        return 7 * self.footprint_elems(pb) * self.esize

    def budget_bytes(self) -> int:
        return 7 * self.plane * self.esize

    def try_admit(self, sc: Scenario) -> bool:
        if not self.free_slots:
            return False
        got = self.alloc.alloc(self.footprint_elems(sc.grid))
        if got is None:
            return False
        sc.off, sc.span = got
        sc.slot = self.free_slots.pop(0)
        self._upload(sc)
        sc.state = "active"
        self.active.append(sc)
        self.table_dirty = True
        return True

    def _patch(self, sc: Scenario) -> L.swe_patch:
        pb = sc.grid
        return L.patch(pb.mx, pb.my, _round_up(pb.mx + 4, 16), pb.dx, pb.dy, off=sc.off,
                       plane_stride=self.plane, group=sc.slot, tref=1, bc=pb.bc)

    def _upload(self, sc: Scenario) -> None:
        """Initial state of an admitted scenario into its pool range: FP64
        planes staged on the device (copied from pinned host arrays, or built
        there from the scenario's parameters), converted into the pool's
        precision by swe_state_import; then its first dt from a speed scan."""
        pb = sc.grid
        pitch = _round_up(pb.mx + 4, 16)
        rows = pb.my + 4
        n = pitch * rows
        inner = (slice(2, pb.my + 2), slice(2, pb.mx + 2))
        dev = torch.zeros(4 * n, dtype=torch.float64, device=self.dev)
        planes = dev.view(4, rows, pitch)
        if sc.problem is not None:
            stage = self.host_f64.get(4 * n)
            stage.zero_()
            hp = stage.view(4, rows, pitch).numpy()
            hp[0][inner] = pb.h
            hp[1][inner] = pb.hu
            hp[2][inner] = pb.hv
            hp[3][inner] = pb.b
            self.hold.append((self.host_f64, stage))
            dev.copy_(stage, non_blocking=True)
        else:
            h, b = sc.spec.device_state(self.dev)
            planes[0][inner] = h
            planes[3][inner] = b
        one = self._patch(sc)
        tab_one = self._to_device(patch_table([one]))
        L.swe_state_import(self.p, tab_one.data_ptr(), 1, pb.mx, pb.my, dev.data_ptr(),
                           dev.data_ptr() + 8 * 3 * n, self.pools[self.cur].data_ptr(),
                           self.b.data_ptr(), self.stream, src_shift=sc.off, src_stride=n)
        self.gstatus[2 * sc.slot: 2 * sc.slot + 2].zero_()
        # first dt of this scenario from a speed scan of its own grid: a one-patch
        # table whose patch is group 0 of a one-group reduction into dt[slot]
        one.group = 0
        tab = self._to_device(patch_table([one]))
        self.smax[2 * sc.slot: 2 * sc.slot + 2].zero_()
        L.swe_speed_scan(self.p, tab.data_ptr(), 1, pb.mx, pb.my, self.pools[self.cur].data_ptr(),
                         self.b.data_ptr(), self.smax.data_ptr() + 16 * sc.slot, self.stream)
        dts = self.dt[sc.slot: sc.slot + 1]
        L.swe_cfl_reduce(self.p, tab.data_ptr(), 1, 1, self.smax.data_ptr() + 16 * sc.slot,
                         dts.data_ptr(), self.status.data_ptr(), 0, 1, self.stream)

    def _rebuild(self) -> None:
        pts = [self._patch(sc) for sc in self.active]
        self.table = self._to_device(patch_table(pts))
        plan = L.swe_batched_plan(pts, self.sched)
        self.items = self._to_device(torch.frombuffer(bytearray(bytes(plan.items)),
                                                      dtype=torch.uint8))
        self.tasks = self._to_device(torch.frombuffer(bytearray(bytes(plan.tasks)),
                                                      dtype=torch.uint8))
        self.nitems = plan.nitems
        self.ntasks, self.nplain, self.nsub = plan.ntasks, plan.nplain, plan.nsub
        # a scenario's smax pair lives at its table index (each reduction
        # leaves the pairs at 0 for the next step)
        self.rsmax = torch.zeros(2 * max(len(self.active), 1), dtype=torch.float64,
                                 device=self.dev)
        self.graphs = {}
        self.table_dirty = False

    def _retire(self, sc: Scenario, keep_result: bool = True):
        """Queue the copy of a finished scenario's surface and of its status
        pair, and free its pool range and slot; returns what _finish needs.
        keep_result False (a cancelled scenario) copies nothing."""
        pb = sc.grid
        out = st = None
        if keep_result:
            pitch = _round_up(pb.mx + 4, 16)
            n = pitch * (pb.my + 4)
            q0 = self.pools[self.cur].view(3, self.plane)[0, sc.off: sc.off + n].view(pb.my + 4,
                                                                                     pitch)
            eta = q0[2:-2, 2: pb.mx + 2]
            if self.p.precision == L.F64:
                bb = self.b[sc.off: sc.off + n].view(pb.my + 4, pitch)[2:-2, 2: pb.mx + 2]
                eta = eta + bb
            out = self.host_state.get(pb.mx * pb.my)
            out.view(pb.my, pb.mx).copy_(eta, non_blocking=True)
            st = self.host_status.get(2)
            st.copy_(self.gstatus[2 * sc.slot: 2 * sc.slot + 2], non_blocking=True)
        self.alloc.release(sc.off, sc.span)
        self.free_slots.append(sc.slot)
        self.free_slots.sort()
        self.active.remove(sc)
        self.table_dirty = True
        return sc, out, st

    def _finish(self, results, t0: float) -> list:
        done = []
        for sc, out, st in results:
            sc.finished = time.perf_counter() - t0
            if out is None:  # cancelled while active
                continue
            pb = sc.grid
            eta = out.view(pb.my, pb.mx).numpy().astype(np.float64)
            if self.p.precision != L.F64:
                eta = eta + self.p.sea_level
            # the early-warning product: the final surface, and what the
            # scenario's own steps reported (status bits, depth resets)
            sc.result = {"eta": eta, "status": int(st[0]), "clamps": int(st[1])}
            sc.state = "done"
            self.host_state.put(out)
            self.host_status.put(st)
            done.append(sc)
        return done

    # -- one round ---------------------------------------------------------------
    def round(self, steps: int) -> None:
        mk = markers()
        if self.table_dirty:
            with mk.range("host: plan"):
                self._rebuild()
        with mk.range("host: enqueue"):
            self._enqueue_round(steps)

    def _advance(self, steps: int, stream: int) -> None:
        """The round's steps, each with the CFL rule and the device retake per
        scenario, enqueued by one library call."""
        L.swe_batched_advance(
            self.p, self.table.data_ptr(), len(self.active), self.max_slots,
            self.items.data_ptr(), self.nitems, self.tasks.data_ptr(),
            self.tasks.data_ptr() + L.SWE_TASK_BYTES * (self.ntasks - self.nplain),
            self.nplain, self.nsub, self.pools[0].data_ptr(), self.pools[1].data_ptr(), self.cur,
            0, 3 * self.plane, self.b.data_ptr(), self.dt.data_ptr(), self.rsmax.data_ptr(),
            self.status.data_ptr(), self.gstatus.data_ptr(), self.group_flags.data_ptr(),
            self.retake.data_ptr(), self.pending.data_ptr(), self.queue_ctr.data_ptr(),
            self.sched, steps, stream)

    def _enqueue_round(self, steps: int) -> None:
        # with graphs, a round is captured once per active set and state
        # buffer, and replayed while the set stays the same
        if self.use_graphs:
            key = (self.cur, steps)
            g = self.graphs.get(key)
            if g is None:
                g = torch.cuda.CUDAGraph()
                side = torch.cuda.Stream(self.dev)
                side.wait_stream(torch.cuda.current_stream(self.dev))
                with torch.cuda.graph(g, stream=side):
                    self._advance(steps, side.cuda_stream)
                torch.cuda.current_stream(self.dev).wait_stream(side)
                self.graphs[key] = g
            g.replay()
        else:
            self._advance(steps, self.stream)
        self.cur = (self.cur + steps) % 2
        for sc in self.active:
            sc.steps_done += steps

    def serve(self, requests, warmup: int = 0, log=None, label: str = "serve",
              cancel: dict | None = None, stop_after_rounds: int | None = None,
              resume: dict | None = None, cancel_after_rounds: dict | None = None):
        """Run the request stream.  requests: list of Scenario with arrival
        times in seconds from the start.  A request whose footprint exceeds
        the whole budget is rejected on its own (state "rejected", with the
        reason); cancel maps request ids to times (s from the start) at which
        the request is withdrawn: dropped if still queued, its slot and memory
        freed at the next round boundary if active (state "cancelled");
        cancel_after_rounds does the same after a number of rounds.
        stop_after_rounds: stop after that many rounds and return, under
        "checkpoint", everything needed to continue (the active scenarios'
        stored planes and step sizes, the queue, the requests not yet
        arrived); resume: such a checkpoint, continued in this server (its
        pool offsets and slots may differ: results do not depend on them).
        Returns a summary dict.  The run is one ROCTx range named `label`,
        its host work ranges named "host: ..." (see timeline.py)."""
        with markers().range(label):
            return self._serve(requests, warmup, log, cancel or {}, stop_after_rounds, resume,
                               cancel_after_rounds or {})

    # -- checkpoint / resume -----------------------------------------------------
    def _frame(self, sc: Scenario):
        pb = sc.grid
        n = _round_up(pb.mx + 4, 16) * (pb.my + 4)
        return n

    def checkpoint_active(self) -> list:
        """Host copies of every active scenario's stored planes (state and bed,
        in the pool's precision), step size and status pair (synchronises)."""
        torch.cuda.synchronize(self.dev)
        saved = []
        for sc in self.active:
            n = self._frame(sc)
            planes = self.pools[self.cur].view(3, self.plane)[:, sc.off: sc.off + n].cpu().clone()
            bed = self.b[sc.off: sc.off + n].cpu().clone()
            saved.append({"scenario": sc, "planes": planes, "bed": bed,
                          "dt": float(self.dt[sc.slot].item()),
                          "gstatus": self.gstatus[2 * sc.slot: 2 * sc.slot + 2].cpu().clone()})
        return saved

    def restore_active(self, saved: list) -> None:
        """Admit checkpointed scenarios with their stored planes (no speed scan:
        their step sizes come with them)."""
        for rec in saved:
            sc = rec["scenario"]
            got = self.alloc.alloc(self.footprint_elems(sc.grid))
            if got is None or not self.free_slots:
                raise L.SweError(f"resume: no room for request {sc.rid}")
            sc.off, sc.span = got
            sc.slot = self.free_slots.pop(0)
            n = self._frame(sc)
            self.pools[self.cur].view(3, self.plane)[:, sc.off: sc.off + n].copy_(
                rec["planes"].to(self.dev))
            self.b[sc.off: sc.off + n].copy_(rec["bed"].to(self.dev))
            self.dt[sc.slot] = rec["dt"]
            self.gstatus[2 * sc.slot: 2 * sc.slot + 2].copy_(rec["gstatus"].to(self.dev))
            self.smax[2 * sc.slot: 2 * sc.slot + 2].zero_()
            self.active.append(sc)
        self.table_dirty = True

    def _serve(self, requests, warmup: int, log, cancel: dict, stop_after_rounds, resume,
               cancel_rounds: dict):
        mk = markers()
        pending = sorted(requests, key=lambda r: r.arrival)
        queue: list[Scenario] = []
        done: list[Scenario] = []
        rejected: list[Scenario] = []
        cancelled: list[Scenario] = []
        inflight: deque = deque()  # (event, results, pinned buffers held)
        t_shift = 0.0
        if resume is not None:
            pending = sorted(resume["pending"], key=lambda r: r.arrival)
            queue = list(resume["queue"])
            t_shift = resume["elapsed"]
            self.restore_active(resume["active"])
        t0 = time.perf_counter() - t_shift
        cells = 0
        rounds = 0
        i = 0
        cancel_left = dict(cancel)
        cancel_rounds_left = dict(cancel_rounds)

        def settle(block: bool) -> None:
            ev, results, held = inflight[0]
            if block:
                ev.synchronize()
            elif not ev.query():
                return
            inflight.popleft()
            for pool, buf in held:
                pool.put(buf)
            with mk.range("host: finish"):
                finished = self._finish(results, t0)
            for sc in finished:
                done.append(sc)
                if log:
                    log(f"[serve] request {sc.rid} ({sc.grid.mx}^2) done, latency "
                        f"{(sc.finished - sc.arrival) * 1e3:.1f} ms")

        while i < len(pending) or queue or self.active or inflight:
            now = time.perf_counter() - t0
            while i < len(pending) and pending[i].arrival <= now:
                queue.append(pending[i])
                i += 1
            # withdrawals due by now (by time, or by rounds run)
            for rid, k in list(cancel_rounds_left.items()):
                if rounds >= k:
                    cancel_left[rid] = 0.0
                    del cancel_rounds_left[rid]
            for rid, t in list(cancel_left.items()):
                if t > now:
                    continue
                hit = next((sc for sc in queue if sc.rid == rid), None)
                if hit is not None:
                    queue.remove(hit)
                    hit.state, hit.finished = "cancelled", now
                    cancelled.append(hit)
                    del cancel_left[rid]
                    continue
                hit = next((sc for sc in self.active if sc.rid == rid), None)
                if hit is not None:
                    self._retire(hit, keep_result=False)
                    hit.state, hit.finished = "cancelled", now
                    cancelled.append(hit)
                    del cancel_left[rid]
            # a request larger than the whole budget can never be admitted:
            # reject it alone, with the reason
            for sc in [sc for sc in queue if self.footprint_bytes(sc.grid) > self.budget_bytes()]:
                queue.remove(sc)
                sc.state = "rejected"
                sc.reason = (f"needs {self.footprint_bytes(sc.grid)} bytes of HBM, more than "
                             f"the server's budget of {self.budget_bytes()}")
                rejected.append(sc)
            # admit oldest first while slots and memory allow (later requests
            # pass one that does not fit only with max_bypass_s > 0)
            with mk.range("host: admit"):
                for sc in admit_in_order(queue, self.try_admit, now, self.max_bypass_s):
                    sc.admitted = time.perf_counter() - t0
            if self.active:
                steps = min(self.R, min(sc.nsteps - sc.steps_done for sc in self.active))
                self.round(steps)
                rounds += 1
                cells += steps * sum(sc.grid.mx * sc.grid.my for sc in self.active)
                with mk.range("host: retire"):
                    results = [self._retire(sc) for sc in
                               [sc for sc in self.active if sc.steps_done >= sc.nsteps]]
                ev = torch.cuda.Event()
                ev.record(torch.cuda.current_stream(self.dev))
                inflight.append((ev, results, self.hold))
                self.hold = []
                if stop_after_rounds is not None and rounds >= stop_after_rounds:
                    while inflight:
                        settle(block=True)
                    ckpt = {"active": self.checkpoint_active(), "queue": list(queue),
                            "pending": pending[i:], "elapsed": time.perf_counter() - t0}
                    for rec in ckpt["active"]:
                        self.active.remove(rec["scenario"])
                    self.active = []
                    return {"stopped": True, "checkpoint": ckpt, "done": done,
                            "rejected": rejected, "cancelled": cancelled}
            # stay one round ahead: wait for the older of two queued rounds, or
            # for the last one when nothing else can be queued
            if inflight and (len(inflight) > 1 or not self.active):
                settle(block=True)
            while inflight:
                before = len(inflight)
                settle(block=False)
                if len(inflight) == before:
                    break
            if not self.active and not inflight and not queue and i < len(pending):
                time.sleep(max(0.0, min(0.01, pending[i].arrival - (time.perf_counter() - t0))))
        torch.cuda.synchronize(self.dev)
        total = time.perf_counter() - t0 - t_shift
        lat = np.array([sc.finished - sc.arrival for sc in done if sc.rid >= warmup])
        flags = self.status.cpu().numpy()
        return {"requests": len(done), "measured": int(lat.size),
                "rejected_requests": len(rejected), "cancelled_requests": len(cancelled),
                "p50_ms": float(np.percentile(lat, 50) * 1e3) if lat.size else None,
                "p99_ms": float(np.percentile(lat, 99) * 1e3) if lat.size else None,
                "cell_updates_per_s": cells / total if total > 0 else None, "wall_s": total,
                "status_flags": int(flags[0]), "clamps": int(flags[1]), "done": done,
                "rejected": rejected, "cancelled": cancelled}
