"""Reference AMR level coupling (FP64, plain loops over cells).

TEST INFRASTRUCTURE ONLY (see the package docstring): only tests/ and the
bench's host baseline may use it.

Qin, LeVeque & Motley, Sec. 3 (patches on levels refined by an integer ratio
in space and time; the recursive time integration; the updating process;
refluxing is dropped, as in the paper's GPU code) and its interpolation and
averaging strategies (a sea at rest must stay at rest; away from the shore
the surface elevation is interpolated and averaged, and the depth follows
from it and the bed).  The paper defers the details of both strategies to
other work; the reading here:

fill (ghost cells of a level-(l+1) patch before each of its substeps k, at
time t_n + (k / r) dt_l):
  - a ghost cell over the interior of another patch of the same level takes
    that cell's values (the first such patch in the hierarchy's order);
  - otherwise it takes the values of the level-l cell under it (piecewise
    constant in space), linear in time between that cell's states before and
    after the level-l step, alpha = k / r:
      both states dry            -> h = 0, hu = hv = 0
      else eta = (1 - alpha) (h_old + b_c) + alpha (h_new + b_c)
           h = max(eta - b_f, 0); hu, hv linear in time; hu = hv = 0 if
           h <= drytol (b_c, b_f: bed of the coarse and of the fine cell).
average (level-l cells under a level-(l+1) patch after its r substeps; the
  r x r fine cells over a coarse cell):
      no fine cell wet           -> h = 0, hu = hv = 0
      else eta = mean of (h + b_f) over the wet fine cells,
           h = max(eta - b_c, 0), hu, hv = mean over all r x r fine cells,
           hu = hv = 0 if h <= drytol.
advance(l, dt): step every level-l patch by dt (level 1: physical boundary
  ghosts; finer levels: the filled ghosts); then, if a finer level exists,
  r times: fill its ghosts (alpha = k / r) and advance(l + 1, dt / r);
  then average it onto level l.

Parity unpinned against the paper's own code (it states no formulas); the
tests pin this reading by invariants: a sea at rest stays bitwise at rest, a
hierarchy with ratio 1 reproduces the single-level run, averaging a linear
surface gives the coarse cell-centre value, and the fill on a field whose
every cell differs.
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


class Hierarchy:
    def __init__(self, H, P):
        self.r = H.ratio
        self.P = P
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

    def fill(self, lev, old, alpha):
        """Ghost cells of level lev (>= 2) from the same level or from level
        lev - 1, whose states before and after its step are `old` (copies of
        that level's q arrays, in patch order) and the current ones."""
        r, drytol = self.r, self.P.drytol
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
                    Ic, Jc = I // r, J // r
                    cidx = [k for k, c in enumerate(self.levels[lev - 2]) if c.covers(Ic, Jc)][0]
                    cn = self.levels[lev - 2][cidx]
                    rc, cc = cn.cell(Ic, Jc)
                    qo, qn = old[cidx][rc, cc], cn.q[rc, cc]
                    bc_ = cn.b[rc, cc]
                    bf = f.b[row, col]
                    if qo[0] <= drytol and qn[0] <= drytol:
                        f.q[row, col, :] = 0.0
                        continue
                    eta = (1.0 - alpha) * (qo[0] + bc_) + alpha * (qn[0] + bc_)
                    h = max(eta - bf, 0.0)
                    if h <= drytol:
                        f.q[row, col, :] = (h, 0.0, 0.0)
                    else:
                        f.q[row, col, :] = (h, (1.0 - alpha) * qo[1] + alpha * qn[1],
                                            (1.0 - alpha) * qo[2] + alpha * qn[2])

    def average(self, lev):
        """Level-lev cells under level lev + 1 patches from the fine cells."""
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
        old = [p.q.copy() for p in self.levels[lev - 1]]
        for p in self.levels[lev - 1]:
            if lev == 1:
                ghost_fill(p.g, p.q)
            out, _, clamps, nf = step(self.P, p.g, p.q, p.b, dt)
            assert nf == 0, "non-finite value in the reference AMR run"
            p.q[2:-2, 2:-2] = out[2:-2, 2:-2]
        if lev < len(self.levels):
            for k in range(self.r):
                self.fill(lev + 1, old, k / self.r)
                self.advance(lev + 1, dt / self.r)
            self.average(lev)

    def run(self, dt1, ncoarse):
        for _ in range(ncoarse):
            self.advance(1, dt1)

    def interior(self, lev, k):
        p = self.levels[lev - 1][k]
        return p.q[2:-2, 2:-2].copy()
