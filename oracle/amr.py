"""Reference AMR level coupling (FP64, plain loops over cells).

TEST INFRASTRUCTURE ONLY (see the package docstring): only tests/ and the
bench's host baseline may use it.

Qin, LeVeque & Motley, Sec. 3 (patches on levels refined by an integer ratio
in space and time; the recursive time integration, whose step 2 fills a
finer level's ghost cells from the same level or by interpolation in space
and time from the level below; the updating process; refluxing is dropped,
as in the paper's GPU code) and its interpolation and averaging strategies:
a sea at rest must stay at rest; away from the shoreline the interpolation
is simple linear interpolation and the averaging takes the arithmetic mean
of the surface elevation, the depth following from the surface and the bed;
near the shoreline, where a cell is dry, no strategy keeps both the mass and
a flat surface.  The reading here:

coarse value at a fine cell (I, J) of level l + 1 from level l (ratio r),
  at time t_n + alpha dt_l between that level's states before (old) and
  after (new) its step:
    the fine cell's centre lies at X = (I + 1/2) / r - 1/2,
    Y = (J + 1/2) / r - 1/2 in level-l cell units (level-l centres at whole
    numbers); its bilinear stencil is the level-l cells (i0 + a, j0 + c),
    a, c in {0, 1}, i0 = floor(X), j0 = floor(Y), with weights
    (1 - wx, wx) and (1 - wy, wy), wx = X - i0, wy = Y - j0 (exact binary
    fractions); a stencil cell of weight 0 (ratio 1) is left out;
    linear (away from the shore): every stencil cell lies in the interior of
      a level-l patch and is wet (h > drytol) in both states; then per
      stencil cell eta_k = (1 - alpha)(h_old + b_k) + alpha (h_new + b_k) and
      momenta (1 - alpha) m_old + alpha m_new, combined as
        v = (1 - wy) ((1 - wx) v_00 + wx v_10) + wy ((1 - wx) v_01 + wx v_11),
      h = max(eta - b_f, 0), hu = hv = 0 if h <= drytol;
    constant (near the shore: otherwise): the level-l cell (I // r, J // r)
      under the fine cell alone:
        both states dry -> h = 0, hu = hv = 0
        else eta = (1 - alpha)(h_old + b_c) + alpha (h_new + b_c),
             h = max(eta - b_f, 0), hu, hv linear in time, zeroed when
             h <= drytol (b_c, b_f: bed of the coarse and of the fine cell).
  Bilinear weights are non-negative, so the linear rule creates no new
  extrema, reproduces a linear surface exactly and keeps a sea at rest at
  rest; the constant rule near dry cells keeps a wet surface from being
  interpolated toward the bed of a dry cell.
fill (ghost cells of a level-(l+1) patch before each of its substeps k,
  alpha = k / r):
  - a ghost cell over the interior of another patch of the same level takes
    that cell's values (the first such patch in the hierarchy's order);
  - otherwise the coarse value above.
average (level-l cells under a level-(l+1) patch after its r substeps; the
  r x r fine cells over a coarse cell):
      no fine cell wet           -> h = 0, hu = hv = 0
      else eta = mean of (h + b_f) over the wet fine cells,
           h = max(eta - b_c, 0), hu, hv = mean over all r x r fine cells,
           hu = hv = 0 if h <= drytol.
advance(l, dt): step every level-l patch by dt (level 1: physical boundary
  ghosts; finer levels: the filled ghosts); then, if a finer level exists,
  r times: fill its ghosts (alpha = k / r) and advance(l + 1, dt / r);
  then average it onto level l.  With regridding every b steps, level l + 1
  and finer are regridded (oracle/regrid.py) at the start of every b-th step
  of level l, from level l's state then.
integrate: dt_1 from the CFL condition (Sec. 2) of the whole hierarchy, a
  level-l patch's rate max(sx, sy) / dx_l divided by r^(l - 1) (Sec. 3: the
  level steps dt_1 / r^(l - 1)); the first dt_1 from a speed scan, each next
  one cfl_desired over the largest rate of the coarse step before; a coarse
  step above cfl_max is redone from a snapshot of every level with the
  reduced dt_1.

Parity unpinned against the paper's own code (it states no formulas); the
tests pin this reading: a sea at rest stays bitwise at rest, a hierarchy with
ratio 1 reproduces the single-level run, a linear surface and linear momenta
are interpolated exactly away from the shore, a dry stencil cell falls back
to the cell under the ghost, averaging a linear surface gives the coarse
cell-centre value.
"""
from __future__ import annotations

import numpy as np

from . import BC_USER, ghost_fill, ghost_fill_b, grid, new_state, step


class OPatch:
    def __init__(self, p, level_dx, bc):
        self.level, self.i0, self.j0, self.mx, self.my = p.level, p.i0, p.j0, p.mx, p.my
        self.q, _ = new_state(p.h, p.hu, p.hv, p.b_frame[2:-2, 2:-2])
        self.b = np.array(p.b_frame, dtype=np.float64)
        self.g = grid(p.mx, p.my, level_dx, level_dx, bc)

    def covers(self, I, J):
        return self.i0 <= I < self.i0 + self.mx and self.j0 <= J < self.j0 + self.my

    def cell(self, I, J):
        """(row, column) of global cell (I, J) in this patch's ghost-framed arrays."""
        return J - self.j0 + 2, I - self.i0 + 2


def coarse_value(coarse, old, r, drytol, alpha, I, J, bf):
    """(h, hu, hv) at fine cell (I, J) of the level above the patches `coarse`
    (OPatch objects, ratio r), with bed bf, at time alpha between `old` (their
    q arrays before their step, in patch order) and their current states; the
    reading in the module docstring."""

    def states(Ic, Jc):
        """(old, new, bed) of the coarse cell (Ic, Jc), or None where no
        coarse patch has it in its interior."""
        for k, c in enumerate(coarse):
            if c.covers(Ic, Jc):
                rc, cc = c.cell(Ic, Jc)
                return old[k][rc, cc], c.q[rc, cc], c.b[rc, cc]
        return None

    X = (I + 0.5) / r - 0.5
    Y = (J + 0.5) / r - 0.5
    i0, j0 = int(np.floor(X)), int(np.floor(Y))
    wx, wy = X - i0, Y - j0
    # (offset, weight) along each axis; a weight of 0 (ratio 1) drops the cell
    cols = [(0, 1.0 - wx)] + ([(1, wx)] if wx > 0.0 else [])
    rows = [(0, 1.0 - wy)] + ([(1, wy)] if wy > 0.0 else [])
    cells = {(a, c): states(i0 + a, j0 + c) for c, _ in rows for a, _ in cols}
    linear = all(st is not None and st[0][0] > drytol and st[1][0] > drytol
                 for st in cells.values())
    if linear:
        v = {}
        for k, (qo, qn, bk) in cells.items():
            v[k] = ((1.0 - alpha) * (qo[0] + bk) + alpha * (qn[0] + bk),
                    (1.0 - alpha) * qo[1] + alpha * qn[1],
                    (1.0 - alpha) * qo[2] + alpha * qn[2])

        def combine(m):
            total = None
            for c, wr in rows:
                line = None
                for a, wc in cols:
                    t = wc * v[a, c][m]
                    line = t if line is None else line + t
                t = wr * line
                total = t if total is None else total + t
            return total
        eta, hu, hv = combine(0), combine(1), combine(2)
    else:
        qo, qn, bc_ = states(I // r, J // r)
        if qo[0] <= drytol and qn[0] <= drytol:
            return (0.0, 0.0, 0.0)
        eta = (1.0 - alpha) * (qo[0] + bc_) + alpha * (qn[0] + bc_)
        hu = (1.0 - alpha) * qo[1] + alpha * qn[1]
        hv = (1.0 - alpha) * qo[2] + alpha * qn[2]
    h = max(eta - bf, 0.0)
    if h <= drytol:
        return (h, 0.0, 0.0)
    return (h, hu, hv)


def _locate(patches, I, J, skip=None):
    """Index (in `patches`) of the first patch whose interior holds each of
    the cells (I, J), -1 where none does; `skip` is left out."""
    k = np.full(I.shape, -1, dtype=np.int64)
    if I.size == 0:
        return k
    lo_i, hi_i, lo_j, hi_j = I.min(), I.max(), J.min(), J.max()
    for n, p in enumerate(patches):
        # a patch clear of the cells' bounding box holds none of them
        if p is skip or p.i0 > hi_i or p.i0 + p.mx <= lo_i or p.j0 > hi_j or p.j0 + p.my <= lo_j:
            continue
        m = (k < 0) & (I >= p.i0) & (I < p.i0 + p.mx) & (J >= p.j0) & (J < p.j0 + p.my)
        k[m] = n
    return k


def _gather(patches, arrays, k, I, J, ncomp):
    """Values of arrays[k] (each a patch's ghost-framed array) at the cells
    (I, J) of patch k; NaN where k < 0."""
    out = np.full(I.shape + ((ncomp,) if ncomp else ()), np.nan)
    for n in np.unique(k[k >= 0]):
        p = patches[n]
        m = k == n
        out[m] = arrays[n][J[m] - p.j0 + 2, I[m] - p.i0 + 2]
    return out


def _max0(d):
    """max(d, 0.0) as Python's max evaluates it (d unless 0.0 > d)."""
    return np.where(0.0 > d, 0.0, d)


def coarse_values(coarse, old, r, drytol, alpha, I, J, bf):
    """coarse_value for arrays of fine cells (I, J) with beds bf: the same
    reading, each value computed by the same operations in the same order
    (numpy float64 arithmetic, element by element).  Returns (h, hu, hv)."""
    X = (I.astype(np.float64) + 0.5) / r - 0.5
    Y = (J.astype(np.float64) + 0.5) / r - 0.5
    i0 = np.floor(X).astype(np.int64)
    j0 = np.floor(Y).astype(np.int64)
    wx, wy = X - i0, Y - j0
    use_x, use_y = wx > 0.0, wy > 0.0
    new = [c.q for c in coarse]
    beds = [c.b for c in coarse]
    v, linear = {}, np.ones(I.shape, dtype=bool)
    for c_ in (0, 1):
        for a in (0, 1):
            used = np.ones(I.shape, dtype=bool)
            if a:
                used &= use_x
            if c_:
                used &= use_y
            k = _locate(coarse, i0 + a, j0 + c_)
            qo = _gather(coarse, old, k, i0 + a, j0 + c_, 3)
            qn = _gather(coarse, new, k, i0 + a, j0 + c_, 3)
            bk = _gather(coarse, beds, k, i0 + a, j0 + c_, 0)
            ok = (k >= 0) & (qo[..., 0] > drytol) & (qn[..., 0] > drytol)
            linear &= ~used | ok
            v[a, c_] = ((1.0 - alpha) * (qo[..., 0] + bk) + alpha * (qn[..., 0] + bk),
                        (1.0 - alpha) * qo[..., 1] + alpha * qn[..., 1],
                        (1.0 - alpha) * qo[..., 2] + alpha * qn[..., 2])
    lin = []
    for m in range(3):
        line0 = (1.0 - wx) * v[0, 0][m]
        line0 = np.where(use_x, line0 + wx * v[1, 0][m], line0)
        line1 = (1.0 - wx) * v[0, 1][m]
        line1 = np.where(use_x, line1 + wx * v[1, 1][m], line1)
        total = (1.0 - wy) * line0
        lin.append(np.where(use_y, total + wy * line1, total))
    # near the shore: the cell under the fine cell alone
    Ic, Jc = I // r, J // r
    k = _locate(coarse, Ic, Jc)
    qo = _gather(coarse, old, k, Ic, Jc, 3)
    qn = _gather(coarse, new, k, Ic, Jc, 3)
    bc_ = _gather(coarse, beds, k, Ic, Jc, 0)
    const = ((1.0 - alpha) * (qo[..., 0] + bc_) + alpha * (qn[..., 0] + bc_),
             (1.0 - alpha) * qo[..., 1] + alpha * qn[..., 1],
             (1.0 - alpha) * qo[..., 2] + alpha * qn[..., 2])
    dry = ~linear & (qo[..., 0] <= drytol) & (qn[..., 0] <= drytol)
    eta = np.where(linear, lin[0], const[0])
    hu = np.where(linear, lin[1], const[1])
    hv = np.where(linear, lin[2], const[2])
    h = _max0(eta - bf)
    wet = h > drytol
    h = np.where(dry, 0.0, h)
    hu = np.where(dry | ~wet, 0.0, hu)
    hv = np.where(dry | ~wet, 0.0, hv)
    return h, hu, hv


class Hierarchy:
    def __init__(self, H, P):
        self.r = H.ratio
        self.P = P
        self.H = H
        self.regrid_every = None
        self.regrid_kw = {}
        self.steps_taken = {}
        self.regrids = []  # (level whose flags drove it, its step count)
        self.levels = []
        for lev in range(1, H.levels() + 1):
            bc = H.bc if lev == 1 else (BC_USER,) * 4
            ps = [OPatch(p, H.dx(lev), bc) for p in H.patches if p.level == lev]
            self.levels.append(ps)
        for p in self.levels[0]:
            ghost_fill_b(p.g, p.b)

    # -- the reading above, cell by cell --------------------------------------
    def find(self, lev, I, J, skip=None):
        for p in self.levels[lev - 1]:
            if p is not skip and p.covers(I, J):
                return p
        return None

    def coarse_value(self, lev, old, alpha, I, J, bf):
        return coarse_value(self.levels[lev - 1], old, self.r, self.P.drytol, alpha, I, J, bf)

    def fill(self, lev, old, alpha):
        """Ghost cells of level lev (>= 2) from the same level or from level
        lev - 1, whose states before and after its step are `old` (copies of
        that level's q arrays, in patch order) and the current ones: the rule
        of fill_cellwise, evaluated for a patch's ghost cells at once (the
        same operations per cell; each ghost cell reads interior cells only,
        so the order in which they are written does not matter)."""
        same = self.levels[lev - 1]
        for f in same:
            rows, cols = np.meshgrid(np.arange(f.my + 4), np.arange(f.mx + 4), indexing="ij")
            ghost = ~((rows >= 2) & (rows < f.my + 2) & (cols >= 2) & (cols < f.mx + 2))
            rows, cols = rows[ghost], cols[ghost]
            I = (f.i0 + cols - 2).astype(np.int64)
            J = (f.j0 + rows - 2).astype(np.int64)
            k = _locate(same, I, J, skip=f)
            cp = k >= 0
            if cp.any():
                f.q[rows[cp], cols[cp]] = _gather(same, [p.q for p in same], k[cp], I[cp], J[cp], 3)
            cv = ~cp
            if cv.any():
                h, hu, hv = coarse_values(self.levels[lev - 2], old, self.r, self.P.drytol, alpha,
                                          I[cv], J[cv], f.b[rows[cv], cols[cv]])
                f.q[rows[cv], cols[cv]] = np.stack([h, hu, hv], axis=-1)

    def fill_cellwise(self, lev, old, alpha):
        """fill, one ghost cell at a time (the reading written out)."""
        for f in self.levels[lev - 1]:
            for row in range(f.my + 4):
                for col in range(f.mx + 4):
                    if 2 <= row < f.my + 2 and 2 <= col < f.mx + 2:
                        continue
                    I, J = f.i0 + col - 2, f.j0 + row - 2
                    s = self.find(lev, I, J, skip=f)
                    if s is not None:
                        f.q[row, col, :] = s.q[s.cell(I, J)]
                        continue
                    f.q[row, col, :] = self.coarse_value(lev - 1, old, alpha, I, J,
                                                         f.b[row, col])

    def average(self, lev):
        """Level-lev cells under level lev + 1 patches from the fine cells:
        the rule of average_cellwise for all coarse cells under a fine patch
        at once (the sums taken over the fine cells in the same order)."""
        r, drytol = self.r, self.P.drytol
        coarse = self.levels[lev - 1]
        for f in self.levels[lev]:
            Jc, Ic = np.meshgrid(np.arange(f.j0 // r, (f.j0 + f.my) // r),
                                 np.arange(f.i0 // r, (f.i0 + f.mx) // r), indexing="ij")
            Ic, Jc = Ic.ravel().astype(np.int64), Jc.ravel().astype(np.int64)
            k = _locate(coarse, Ic, Jc)
            seta = np.zeros(Ic.shape)
            nwet = np.zeros(Ic.shape, dtype=np.int64)
            hu = np.zeros(Ic.shape)
            hv = np.zeros(Ic.shape)
            for dj in range(r):
                for di in range(r):
                    rf = Jc * r + dj - f.j0 + 2
                    cf = Ic * r + di - f.i0 + 2
                    h = f.q[rf, cf, 0]
                    wet = h > drytol
                    seta = np.where(wet, seta + (h + f.b[rf, cf]), seta)
                    nwet += wet
                    hu = hu + f.q[rf, cf, 1]
                    hv = hv + f.q[rf, cf, 2]
            bc_ = _gather(coarse, [c.b for c in coarse], k, Ic, Jc, 0)
            any_wet = nwet > 0
            eta = seta / np.maximum(nwet, 1)
            hc = _max0(eta - bc_)
            keep = any_wet & (hc > drytol)
            out = np.stack([np.where(any_wet, hc, 0.0), np.where(keep, hu / (r * r), 0.0),
                            np.where(keep, hv / (r * r), 0.0)], axis=-1)
            for n, c in enumerate(coarse):
                m = k == n
                if m.any():
                    c.q[Jc[m] - c.j0 + 2, Ic[m] - c.i0 + 2] = out[m]

    def average_cellwise(self, lev):
        """average, one coarse cell at a time (the reading written out)."""
        r, drytol = self.r, self.P.drytol
        for f in self.levels[lev]:
            for Jc in range(f.j0 // r, (f.j0 + f.my) // r):
                for Ic in range(f.i0 // r, (f.i0 + f.mx) // r):
                    c = self.find(lev, Ic, Jc)
                    rc, cc = c.cell(Ic, Jc)
                    etas, hu, hv = [], 0.0, 0.0
                    for dj in range(r):
                        for di in range(r):
                            rf, cf = f.cell(Ic * r + di, Jc * r + dj)
                            h = f.q[rf, cf, 0]
                            if h > drytol:
                                etas.append(h + f.b[rf, cf])
                            hu += f.q[rf, cf, 1]
                            hv += f.q[rf, cf, 2]
                    if not etas:
                        c.q[rc, cc, :] = 0.0
                        continue
                    eta = sum(etas) / len(etas)
                    h = max(eta - c.b[rc, cc], 0.0)
                    if h <= drytol:
                        c.q[rc, cc, :] = (h, 0.0, 0.0)
                    else:
                        c.q[rc, cc, :] = (h, hu / (r * r), hv / (r * r))

    def advance(self, lev, dt):
        if self.regrid_every and lev < len(self.levels):
            # level lev + 1 and finer regridded every b steps of level lev,
            # from level lev's state at the start of its step (the levels
            # above it are at the same time)
            n = self.steps_taken.get(lev, 0)
            if n > 0 and n % self.regrid_every == 0:
                from .regrid import regrid
                regrid(self, self.H, base=lev, **self.regrid_kw)
                self.regrids.append((lev, n))
        old = [p.q.copy() for p in self.levels[lev - 1]]
        for p in self.levels[lev - 1]:
            if lev == 1:
                ghost_fill(p.g, p.q)
            out, sm, clamps, nf = step(self.P, p.g, p.q, p.b, dt)
            assert nf == 0, "non-finite value in the reference AMR run"
            p.q[2:-2, 2:-2] = out[2:-2, 2:-2]
            p.smax = np.maximum(getattr(p, "smax", np.zeros(2)), sm)
        self.steps_taken[lev] = self.steps_taken.get(lev, 0) + 1
        if lev < len(self.levels):
            for k in range(self.r):
                self.fill(lev + 1, old, k / self.r)
                self.advance(lev + 1, dt / self.r)
            self.average(lev)

    def run(self, dt1, ncoarse):
        for _ in range(ncoarse):
            self.advance(1, dt1)

    # -- step sizes from the CFL condition (Sec. 2; Sec. 3: dt_{l+1} = dt_l / r) ----
    def rate(self):
        """Largest Courant rate of the last coarse step: over the patches of
        every level, max(sx / dx_l, sy / dx_l) / r^(l - 1) (a level-l patch
        steps dt_1 / r^(l - 1)), with (sx, sy) its largest speeds over the
        step's substeps."""
        worst = 0.0
        for lev, ps in enumerate(self.levels, start=1):
            d, tref = self.H.dx(lev), float(self.r ** (lev - 1))
            for p in ps:
                sx, sy = getattr(p, "smax", np.zeros(2))
                v = max(sx / d, sy / d) / tref
                worst = v if v > worst else worst
        return worst

    def reset_speeds(self):
        for ps in self.levels:
            for p in ps:
                p.smax = np.zeros(2)

    def initial_dt(self):
        """dt_1 from the speeds of the initial state (every level's ghost
        cells filled first, the finer ones from the level below at alpha 0)."""
        from . import speed_scan
        self.reset_speeds()
        for lev, ps in enumerate(self.levels, start=1):
            if lev > 1:
                self.fill(lev, [c.q.copy() for c in self.levels[lev - 2]], 0.0)
            for p in ps:
                if lev == 1:
                    ghost_fill(p.g, p.q)
                p.smax = speed_scan(self.P, p.g, p.q, p.b)
        rate = self.rate()
        return self.P.cfl_desired / rate if rate > 0.0 else 1.0

    def snapshot(self):
        import copy
        return ([[copy.copy(p) for p in ps] for ps in self.levels],
                [[p.q.copy() for p in ps] for ps in self.levels], dict(self.steps_taken),
                len(self.regrids))

    def restore(self, snap):
        lists, qs, steps, nreg = snap
        self.levels = [list(ps) for ps in lists]
        for ps, qq in zip(self.levels, qs):
            for p, q in zip(ps, qq):
                p.q = q.copy()
        self.steps_taken = dict(steps)
        del self.regrids[nreg:]

    def integrate(self, ncoarse, regrid_every=None, regrid_kw=None, dt0=None):
        """ncoarse coarse steps with dt_1 from the CFL condition: the first
        from a speed scan, each next one cfl_desired / rate of the step before;
        a coarse step whose Courant number dt_1 rate exceeds cfl_max is redone
        (every level restored, regridding included) with dt_1 = cfl_desired /
        rate.  With regrid_every = b, level l + 1 and finer are regridded every
        b steps of level l (regrid_kw: tol, buffer, efficiency, min_side).
        dt0: the first dt_1 instead of the speed scan's.
        Returns the accepted dt_1 sequence and the number of retakes."""
        self.regrid_every = regrid_every
        self.regrid_kw = dict(regrid_kw or {})
        dt = self.initial_dt() if dt0 is None else float(dt0)
        dts, retakes = [], 0
        for _ in range(ncoarse):
            snap = self.snapshot()
            while True:
                self.reset_speeds()
                self.advance(1, dt)
                rate = self.rate()
                if rate > 0.0 and dt * rate > self.P.cfl_max:
                    self.restore(snap)
                    dt = self.P.cfl_desired / rate
                    retakes += 1
                    continue
                break
            dts.append(dt)
            if rate > 0.0:
                dt = self.P.cfl_desired / rate
        self.regrid_every = None
        return np.array(dts), retakes

    def interior(self, lev, k):
        p = self.levels[lev - 1][k]
        return p.q[2:-2, 2:-2].copy()
