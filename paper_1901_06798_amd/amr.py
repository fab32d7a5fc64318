"""A nested AMR hierarchy advanced on the device (Qin, LeVeque & Motley,
Sec. 3: levels refined by an integer ratio r in space and time, the recursive
time integration, ghost cells of a finer level from the same level or from
the level below, the updating process; refluxing is left out, as in the
paper's GPU code).

Each level is one BatchedSolver: its patches live in one pool (two state
buffers and the bed), and a level step is one swe_batched_step.  Patches of
level 2 and finer have user boundaries on every side: their ghost cells are
written by swe_amr_fill before each of their substeps.  The fill and averaging
plans (which cell each ghost cell or covered coarse cell reads) are built on
the device from the levels' rectangles, once per set of patches; a coarse
step is then a fixed sequence of launches, with the step sizes in device
memory, that can be captured into a HIP graph.

Nesting required (not checked cell by cell): every ghost cell of a level-l
patch (l >= 2) lies over an interior cell of the same level or of level
l - 1; patches of one level do not overlap; a finer patch's extents are
multiples of r in its level's index.
"""
from __future__ import annotations

import numpy as np
import torch

from . import _lib as L
from .batched import BatchedSolver
from .workloads import BC_USER, AmrHierarchy, Problem

FILL_DTYPE = np.dtype([("dst", "<i8"), ("src", "<i8"), ("st", "<i8", (4,)), ("wx", "<f8"),
                       ("wy", "<f8"), ("kind", "<i4"), ("reserved", "<i4")])
AVG_DTYPE = np.dtype([("dst", "<i8"), ("src", "<i8"), ("pitch", "<i4"), ("reserved", "<i4")])


class _Geo:
    """Where a level's patches sit: global index origin and pool layout."""

    def __init__(self, patches, bs: BatchedSolver):
        self.i0 = np.array([p.i0 for p in patches])
        self.j0 = np.array([p.j0 for p in patches])
        self.mx = np.array([p.mx for p in patches])
        self.my = np.array([p.my for p in patches])
        self.off = np.array(bs.offs, dtype=np.int64)
        self.pitch = np.array([lay[0] for lay in bs.layout], dtype=np.int64)

    def covering(self, I, J, skip: int = -1):
        """Index of the first patch whose interior holds (I, J), else -1."""
        out = np.full(I.shape, -1, dtype=np.int64)
        for k in range(len(self.i0)):
            if k == skip:
                continue
            m = ((out < 0) & (I >= self.i0[k]) & (I < self.i0[k] + self.mx[k])
                 & (J >= self.j0[k]) & (J < self.j0[k] + self.my[k]))
            out[m] = k
        return out

    def elem(self, k, I, J):
        """Element offset of global cell (I, J) in patch k's planes."""
        return (self.off[k] + (J - self.j0[k] + 2) * self.pitch[k] + (I - self.i0[k] + 2))

    def rects(self, dev) -> torch.Tensor:
        """The level's swe_amr_rect table, on the device."""
        t = np.zeros(len(self.i0), dtype=L.AMR_RECT_DTYPE)
        t["off"], t["i0"], t["j0"] = self.off, self.i0, self.j0
        t["mx"], t["my"], t["pitch"] = self.mx, self.my, self.pitch
        return torch.from_numpy(t.view(np.uint8)).to(dev)


def stencil(coarse: _Geo, I: np.ndarray, J: np.ndarray, r: int):
    """Bilinear stencil on the level below (ratio r) of the fine cells (I, J):
    the fine centre lies at X = (I + 1/2) / r - 1/2, Y = (J + 1/2) / r - 1/2
    in coarse cell units; the stencil is the coarse cells (i0 + a, j0 + c),
    i0 = floor(X), j0 = floor(Y), in the order (0, 0), (1, 0), (0, 1), (1, 1),
    with weights wx = X - i0, wy = Y - j0.  Returns (st, wx, wy): st[:, k] is
    the element offset of stencil cell k in the first patch of `coarse` whose
    interior holds it, -1 where none does."""
    X = (I + 0.5) / r - 0.5
    Y = (J + 0.5) / r - 0.5
    i0 = np.floor(X).astype(np.int64)
    j0 = np.floor(Y).astype(np.int64)
    wx, wy = X - i0, Y - j0
    st = np.full((I.size, 4), -1, dtype=np.int64)
    for k, (a, c) in enumerate(((0, 0), (1, 0), (0, 1), (1, 1))):
        Ic, Jc = i0 + a, j0 + c
        who = coarse.covering(Ic, Jc)
        for c_ in np.unique(who[who >= 0]):
            m = who == c_
            st[m, k] = coarse.elem(c_, Ic[m], Jc[m])
    return st, wx, wy


def fill_plan(fine: _Geo, coarse: _Geo, r: int) -> np.ndarray:
    ops = []
    for k in range(len(fine.i0)):
        rows, cols = np.meshgrid(np.arange(fine.my[k] + 4), np.arange(fine.mx[k] + 4),
                                 indexing="ij")
        ghost = ~((rows >= 2) & (rows < fine.my[k] + 2) & (cols >= 2) & (cols < fine.mx[k] + 2))
        rows, cols = rows[ghost], cols[ghost]
        I = fine.i0[k] + cols - 2
        J = fine.j0[k] + rows - 2
        dst = fine.off[k] + rows * fine.pitch[k] + cols
        same = fine.covering(I, J, skip=k)
        Ic, Jc = I // r, J // r
        below = coarse.covering(Ic, Jc)
        if np.any((same < 0) & (below < 0)):
            raise L.SweError(f"patch {k}: a ghost cell lies over no cell of its level or the "
                             f"level below")
        op = np.zeros(dst.size, dtype=FILL_DTYPE)
        op["dst"] = dst
        cp = same >= 0
        for s in np.unique(same[cp]):
            m = same == s
            op["src"][m] = fine.elem(s, I[m], J[m])
        op["kind"][cp] = L.SWE_AMR_COPY
        for c in np.unique(below[~cp]):
            m = (~cp) & (below == c)
            op["src"][m] = coarse.elem(c, Ic[m], Jc[m])
        op["kind"][~cp] = L.SWE_AMR_COARSE
        op["st"] = -1
        if (~cp).any():
            st, wx, wy = stencil(coarse, I[~cp], J[~cp], r)
            op["st"][~cp], op["wx"][~cp], op["wy"][~cp] = st, wx, wy
        ops.append(op)
    return np.concatenate(ops) if ops else np.zeros(0, dtype=FILL_DTYPE)


def average_plan(fine: _Geo, coarse: _Geo, r: int) -> np.ndarray:
    ops = []
    for k in range(len(fine.i0)):
        jc = np.arange(fine.j0[k] // r, (fine.j0[k] + fine.my[k]) // r)
        ic = np.arange(fine.i0[k] // r, (fine.i0[k] + fine.mx[k]) // r)
        Jc, Ic = np.meshgrid(jc, ic, indexing="ij")
        Jc, Ic = Jc.ravel(), Ic.ravel()
        below = coarse.covering(Ic, Jc)
        if np.any(below < 0):
            raise L.SweError(f"patch {k}: not over the level below")
        op = np.zeros(Ic.size, dtype=AVG_DTYPE)
        for c in np.unique(below):
            m = below == c
            op["dst"][m] = coarse.elem(c, Ic[m], Jc[m])
        op["src"] = fine.elem(k, Ic * r, Jc * r)
        op["pitch"] = fine.pitch[k]
        ops.append(op)
    return np.concatenate(ops) if ops else np.zeros(0, dtype=AVG_DTYPE)


class AmrSolver:
    def __init__(self, H: AmrHierarchy, params: L.swe_params | None = None,
                 device: str = "cuda:0", rows=None):
        self.H = H
        self.p = params or L.params()
        self.r = H.ratio
        self.dev = torch.device(device)
        self.nlev = H.levels()
        # 8-row tasks: a level's launch then holds enough waves to fill the
        # device (32-row tasks left most wave slots idle and were 1.6 x slower
        # on the bench hierarchy)
        self.rows = list(rows) if rows is not None else [8] * self.nlev
        self.levels, self.geo, self.lpatches = [], [], []
        for lev in range(1, self.nlev + 1):
            ps = [p for p in H.patches if p.level == lev]
            bs = self._level_solver(lev, ps)
            self.levels.append(bs)
            self.lpatches.append(ps)
            self.geo.append(_Geo(ps, bs))
        self._plans()
        self.dts = torch.zeros(self.nlev, dtype=torch.float64, device=self.dev)
        self.dt1 = torch.zeros(1, dtype=torch.float64, device=self.dev)
        self.cfl_status = torch.zeros(2, dtype=torch.int32, device=self.dev)
        self.cfl_retake = torch.zeros(1, dtype=torch.int32, device=self.dev)
        self.steps_taken = {}
        self.regrid_every = None
        self.regrid_kw = {}
        self.regrids = []
        self._speeds()
        self.graph = None

    def _level_solver(self, lev: int, ps, fresh: bool = False) -> BatchedSolver:
        """The level's pool.  fresh: patches made by regridding, whose cells
        swe_amr_init writes: only their bed is uploaded."""
        bc = self.H.bc if lev == 1 else (BC_USER,) * 4
        d = self.H.dx(lev)
        probs = [Problem(f"l{lev}p{k}", p.h, p.hu, p.hv, p.b_frame[2:-2, 2:-2], d, d, bc,
                         meta={"level": lev}) for k, p in enumerate(ps)]
        bs = BatchedSolver(probs, self.p,
                           sched=L.schedule(seg=64, rows_per_task=self.rows[lev - 1]),
                           device=self.dev, upload=not fresh)
        if lev > 1:  # the bed of the ghost frame (user sides are read from memory)
            for k, p in enumerate(ps):
                bs._view(bs.b, k, 1)[0][:, : p.mx + 4] = torch.from_numpy(
                    np.ascontiguousarray(p.b_frame)).to(self.dev)
        return bs

    def _plans(self) -> None:
        """The ghost-fill and averaging plans of every level above the first,
        built on the device from the levels' rectangle tables (swe_amr_plans;
        fill_plan and average_plan build the same on the host)."""
        self.fill_ops, self.avg_ops, self.nfill, self.navg = [None], [], [0], []
        r = self.r
        for lev in range(1, self.nlev):
            fine, coarse = self.geo[lev], self.geo[lev - 1]
            mx, my = fine.mx.astype(np.int64), fine.my.astype(np.int64)
            i0, j0 = fine.i0.astype(np.int64), fine.j0.astype(np.int64)
            ng = (mx + 4) * (my + 4) - mx * my
            na = ((i0 + mx) // r - i0 // r) * ((j0 + my) // r - j0 // r)
            ff = np.concatenate([[0], np.cumsum(ng)[:-1]]).astype(np.int64)
            af = np.concatenate([[0], np.cumsum(na)[:-1]]).astype(np.int64)
            fill = torch.empty(int(ng.sum()) * FILL_DTYPE.itemsize, dtype=torch.uint8,
                               device=self.dev)
            avg = torch.empty(int(na.sum()) * AVG_DTYPE.itemsize, dtype=torch.uint8,
                              device=self.dev)
            tf, tc = fine.rects(self.dev), coarse.rects(self.dev)
            firsts = torch.from_numpy(np.concatenate([ff, af])).to(self.dev)
            err = torch.zeros(1, dtype=torch.int32, device=self.dev)
            L.swe_amr_plans(tf.data_ptr(), len(fine.i0), tc.data_ptr(), len(coarse.i0), r,
                            int((ng + na).max()), fill.data_ptr(), firsts.data_ptr(),
                            avg.data_ptr(), firsts.data_ptr() + 8 * len(ff), err.data_ptr(),
                            self.stream)
            e = int(err.item())  # waits for the plans (and keeps the tables alive until then)
            if e & 1:
                raise L.SweError(f"level {lev + 1}: a ghost cell lies over no cell of its level "
                                 f"or the level below")
            if e & 2:
                raise L.SweError(f"level {lev + 1}: a patch is not over the level below")
            self.fill_ops.append(fill)
            self.avg_ops.append(avg)
            self.nfill.append(int(ng.sum()))
            self.navg.append(int(na.sum()))

    # -- regridding --------------------------------------------------------------
    def refine_flags(self, lev: int, tol: float = 5e-3, buffer: int = 2) -> torch.Tensor:
        """Refinement flags of level lev (device uint8 plane, the level's layout)."""
        bs = self.levels[lev - 1]
        margin = 2 if self.r == 1 else 1
        out = torch.zeros(bs.plane, dtype=torch.uint8, device=self.dev)
        L.swe_amr_flag(self.p, bs.table.data_ptr(), bs.n, bs.max_mx, bs.max_my,
                       bs.pools[bs.cur].data_ptr(), bs.b.data_ptr(), tol, buffer, margin,
                       out.data_ptr(), self.stream)
        return out

    def regrid(self, tol: float = 5e-3, buffer: int = 2, efficiency: float = 0.7,
               min_side: int = 2, base: int = 1) -> list:
        """Regrid the levels above `base` from the current state (levels base
        and finer synchronised):
        flags on the device, clustering on the host, new patches filled on the
        device from the old ones of their level where those overlap, else from
        the level below (which is regridded first).  Host work; returns the
        new rectangles (i0, j0, mx, my) per level."""
        import time

        from .workloads import AmrPatch
        r = self.r
        t_start = time.perf_counter()
        t_flag = t_cluster = t_pool = 0.0
        for lev in range(base + 1, self.nlev + 1):
            parent, pps = self.levels[lev - 2], self.lpatches[lev - 2]
            t0 = time.perf_counter()
            fh = self.refine_flags(lev - 1, tol, buffer).cpu().numpy()
            t1 = time.perf_counter()
            rects = []
            for k, p in enumerate(pps):
                pitch, off = parent.layout[k][0], parent.offs[k]
                F = fh[off: off + pitch * (p.my + 4)].reshape(p.my + 4, pitch)
                for (a, b_, c, d) in L.swe_amr_cluster(F[2: p.my + 2, 2: p.mx + 2],
                                                       efficiency, min_side):
                    rects.append(((p.i0 + a) * r, (p.j0 + b_) * r, (c - a + 1) * r,
                                  (d - b_ + 1) * r))
            t_flag += t1 - t0
            t_cluster += time.perf_counter() - t1
            if not rects:  # nothing to refine: this level and the finer ones end
                self.nlev = lev - 1
                del self.levels[lev - 1:], self.geo[lev - 1:], self.lpatches[lev - 1:]
                del self.rows[lev - 1:]
                break
            t2 = time.perf_counter()
            new_ps = []
            for (i0, j0, mx, my) in rects:
                z = np.zeros((my, mx))
                new_ps.append(AmrPatch(lev, i0, j0, mx, my, z, z, z,
                                       self.H.bed_frame(lev, i0, j0, mx, my)))
            bs = self._level_solver(lev, new_ps, fresh=True)
            geo = _Geo(new_ps, bs)
            old_bs, old_geo = self.levels[lev - 1], self.geo[lev - 1]
            t3 = time.perf_counter()
            t_pool += t3 - t2
            cgeo = self.geo[lev - 2]
            tn, to, tc = geo.rects(self.dev), old_geo.rects(self.dev), cgeo.rects(self.dev)
            L.swe_amr_init(self.p, r, tn.data_ptr(), len(new_ps),
                           int(max(p.mx * p.my for p in new_ps)), bs.pools[bs.cur].data_ptr(),
                           bs.plane, bs.b.data_ptr(), to.data_ptr(), len(old_geo.i0),
                           old_bs.pools[old_bs.cur].data_ptr(), old_bs.plane, tc.data_ptr(),
                           len(cgeo.i0), parent.pools[parent.cur].data_ptr(), parent.plane,
                           parent.b.data_ptr(), self.stream)
            torch.cuda.synchronize(self.dev)  # the tables and the old level are released
            self.levels[lev - 1], self.geo[lev - 1], self.lpatches[lev - 1] = bs, geo, new_ps
        self._plans()
        self.dts = self.dts[: self.nlev].clone()
        self._speeds(keep_levels=base)
        self.graph = None
        torch.cuda.synchronize(self.dev)
        total = time.perf_counter() - t_start
        # wall-clock phases of this regrid: flags (device, with the copy to the
        # host), clustering (host), new pools with their bed, and the fill of
        # the new cells with the coupling plans
        self.last_regrid_ms = {"total": 1e3 * total, "flags": 1e3 * t_flag,
                               "cluster": 1e3 * t_cluster, "pools": 1e3 * t_pool,
                               "fill_and_plans": 1e3 * (total - t_flag - t_cluster - t_pool)}
        return [[(p.i0, p.j0, p.mx, p.my) for p in ps] for ps in self.lpatches]

    # -- CFL condition over the hierarchy (Sec. 2; Sec. 3: dt_{l+1} = dt_l / r) --
    def _speeds(self, keep_levels: int = 0) -> None:
        """One speed array for every patch of every level (each level's
        batched step max-combines into its slice) and a patch table of the
        whole hierarchy for swe_cfl_reduce: one group, a level-l patch with
        its dx and tref = r^(l - 1).  The speeds of the first keep_levels
        levels are carried over (a regrid replaced only the finer ones)."""
        old = [bs.smax for bs in self.levels[:keep_levels]]
        total = sum(bs.n for bs in self.levels)
        self.smax_all = torch.zeros(2 * max(total, 1), dtype=torch.float64, device=self.dev)
        pts, k = [], 0
        for lev, bs in enumerate(self.levels, start=1):
            view = self.smax_all[2 * k: 2 * (k + bs.n)]
            if lev <= keep_levels:
                view.copy_(old[lev - 1])
            bs.smax = view
            for pt in bs.patches:
                q = L.patch(pt.mx, pt.my, pt.pitch, pt.dx, pt.dy, off=pt.off,
                            plane_stride=pt.plane_stride, group=0, tref=self.r ** (lev - 1),
                            level=lev, bc=tuple(pt.bc))
                pts.append(q)
            k += bs.n
        from .solver import patch_table
        self.cfl_table = patch_table(pts).to(self.dev)
        self.cfl_n = len(pts)

    def _reduce(self, initial: bool, retake: bool) -> None:
        """dt_1 from the speeds of the whole hierarchy, then every level's step."""
        L.swe_cfl_reduce(self.p, self.cfl_table.data_ptr(), self.cfl_n, 1,
                         self.smax_all.data_ptr(), self.dt1.data_ptr(),
                         self.cfl_status.data_ptr(), 0, 1 if initial else 0, self.stream,
                         retake=self.cfl_retake.data_ptr() if retake else 0)
        L.swe_level_steps(self.dt1.data_ptr(), self.r, self.nlev, self.dts.data_ptr(),
                          self.stream)

    def initial_dt(self) -> float:
        """dt_1 from the speeds of the current state: the ghost cells of every
        finer level filled from the level below at alpha 0, then a speed scan
        of every patch."""
        self.smax_all.zero_()
        for lev in range(1, self.nlev + 1):
            bs = self.levels[lev - 1]
            if lev > 1:
                c = self.levels[lev - 2]
                cur = c.pools[c.cur]
                L.swe_amr_fill(self.p, self.fill_ops[lev - 1].data_ptr(), self.nfill[lev - 1],
                               bs.pools[bs.cur].data_ptr(), bs.plane, bs.b.data_ptr(),
                               cur.data_ptr(), cur.data_ptr(), c.plane, c.b.data_ptr(), 0.0,
                               self.stream)
            L.swe_speed_scan(self.p, bs.table.data_ptr(), bs.n, bs.max_mx, bs.max_my,
                             bs.pools[bs.cur].data_ptr(), bs.b.data_ptr(), bs.smax.data_ptr(),
                             self.stream)
        self._reduce(initial=True, retake=False)
        return float(self.dt1.item())

    def _snapshot(self) -> dict:
        return {"levels": list(self.levels), "geo": list(self.geo),
                "lpatches": list(self.lpatches), "rows": list(self.rows), "nlev": self.nlev,
                "cur": [bs.cur for bs in self.levels],
                "pools": [bs.pools[bs.cur].clone() for bs in self.levels],
                "steps_taken": dict(self.steps_taken), "nregrids": len(self.regrids)}

    def _restore(self, snap: dict) -> None:
        self.levels, self.geo = list(snap["levels"]), list(snap["geo"])
        self.lpatches, self.rows, self.nlev = list(snap["lpatches"]), list(snap["rows"]), snap["nlev"]
        for bs, cur, pool in zip(self.levels, snap["cur"], snap["pools"]):
            bs.cur = cur
            bs.pools[cur].copy_(pool)
        self.steps_taken = dict(snap["steps_taken"])
        del self.regrids[snap["nregrids"]:]
        self._plans()
        self.dts = self.dts[: self.nlev].clone() if self.dts.numel() >= self.nlev else \
            torch.zeros(self.nlev, dtype=torch.float64, device=self.dev)
        self._speeds()
        self.graph = None

    def integrate(self, ncoarse: int, regrid_every: int | None = None, regrid_kw=None,
                  dt0: float | None = None, retake: bool = True) -> tuple:
        """ncoarse coarse steps with dt_1 from the CFL condition of the whole
        hierarchy, computed on the device after each coarse step (the first
        from a speed scan, or dt0); with retake, a coarse step above cfl_max
        is redone from a snapshot of every level (their states and, when a
        regrid happened inside the step, their patches) with the reduced dt_1.
        regrid_every = b: level l + 1 and finer are regridded at the start of
        every b-th step of level l.  Returns the accepted dt_1 values and the
        number of retakes."""
        self.regrid_every = regrid_every
        self.regrid_kw = dict(regrid_kw or {})
        if dt0 is None:
            self.initial_dt()
        else:
            self.dt1.fill_(float(dt0))
            L.swe_level_steps(self.dt1.data_ptr(), self.r, self.nlev, self.dts.data_ptr(),
                              self.stream)
        dts, retakes = [], 0
        try:
            for _ in range(ncoarse):
                snap = self._snapshot() if retake else None
                while True:
                    dt = float(self.dt1.item())
                    self.smax_all.zero_()
                    self._advance(1)
                    self._reduce(initial=False, retake=retake)
                    if retake and int(self.cfl_retake.item()):
                        self._restore(snap)
                        L.swe_level_steps(self.dt1.data_ptr(), self.r, self.nlev,
                                          self.dts.data_ptr(), self.stream)
                        retakes += 1
                        continue
                    break
                dts.append(dt)
        finally:
            self.regrid_every = None
        return np.array(dts), retakes

    @property
    def stream(self) -> int:
        return torch.cuda.current_stream(self.dev).cuda_stream

    def set_dt(self, dt1: float) -> None:
        """Level step sizes dt_l = dt_{l-1} / r."""
        dts = [float(dt1)]
        for _ in range(1, self.nlev):
            dts.append(dts[-1] / self.r)
        self.dts.copy_(torch.tensor(dts, dtype=torch.float64))

    def _advance(self, lev: int) -> None:
        if self.regrid_every and lev < self.nlev:
            n = self.steps_taken.get(lev, 0)
            if n > 0 and n % self.regrid_every == 0:
                self.regrid(base=lev, **self.regrid_kw)
                self.regrids.append((lev, n))
        bs = self.levels[lev - 1]
        old = bs.pools[bs.cur]
        bs.enqueue_step(cfl=False, dt_ptr=self.dts.data_ptr() + 8 * (lev - 1))
        self.steps_taken[lev] = self.steps_taken.get(lev, 0) + 1
        new = bs.pools[bs.cur]
        if lev == self.nlev:
            return
        fine = self.levels[lev]
        for k in range(self.r):
            L.swe_amr_fill(self.p, self.fill_ops[lev].data_ptr(), self.nfill[lev],
                           fine.pools[fine.cur].data_ptr(), fine.plane, fine.b.data_ptr(),
                           old.data_ptr(), new.data_ptr(), bs.plane, bs.b.data_ptr(),
                           k / self.r, self.stream)
            self._advance(lev + 1)
        L.swe_amr_average(self.p, self.avg_ops[lev - 1].data_ptr(), self.navg[lev - 1], self.r,
                          fine.pools[fine.cur].data_ptr(), fine.plane, fine.b.data_ptr(),
                          new.data_ptr(), bs.plane, bs.b.data_ptr(), self.stream)

    def enqueue_coarse_step(self) -> None:
        self._advance(1)

    def run(self, ncoarse: int) -> None:
        for _ in range(ncoarse):
            self._advance(1)

    def capture(self, ncoarse: int = 2) -> None:
        """Capture ncoarse coarse steps into a HIP graph (every level's state
        buffer must come back to where it started: level 1 flips once per
        coarse step, level l r^(l-1) times)."""
        flips = [ncoarse * self.r ** (lev - 1) for lev in range(1, self.nlev + 1)]
        if any(f % 2 for f in flips):
            raise ValueError("capture a number of coarse steps that returns every buffer")
        s = torch.cuda.Stream(self.dev)
        s.wait_stream(torch.cuda.current_stream(self.dev))
        g = torch.cuda.CUDAGraph()
        with torch.cuda.stream(s):
            torch.cuda.synchronize(self.dev)
            with torch.cuda.graph(g, stream=s):
                self.run(ncoarse)
        torch.cuda.current_stream(self.dev).wait_stream(s)
        self.graph = g
        self.graph_steps = ncoarse

    def replay(self) -> None:
        self.graph.replay()

    # -- results ---------------------------------------------------------------
    def state(self, lev: int, k: int):
        """Interior (h, hu, hv) of patch k of level lev."""
        return self.levels[lev - 1].state(k)

    def courant(self) -> float:
        """Largest Courant number over the levels' steps so far (from the speed
        maxima the steps max-combined)."""
        worst = 0.0
        dts = self.dts.cpu().numpy()
        for lev, bs in enumerate(self.levels, start=1):
            sm = bs.smax.cpu().numpy().reshape(-1, 2)
            d = self.H.dx(lev)
            worst = max(worst, float(dts[lev - 1] * max(sm[:, 0].max(), sm[:, 1].max()) / d))
        return worst

    def flags(self):
        f, c = 0, 0
        for bs in self.levels:
            a, b = bs.flags()
            f |= a
            c += b
        return f, c

    def cells_per_coarse_step(self) -> int:
        return sum(p.mx * p.my * self.r ** (p.level - 1) for ps in self.lpatches for p in ps)
