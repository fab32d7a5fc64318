"""Reference regridding of an AMR hierarchy (FP64 states, integer cell work).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Qin, LeVeque & Motley, Sec. 3 (regridding): cells of level l are flagged
where the sea surface departs from rest by more than a tolerance, a buffer
of cells around them is flagged as well, the flags are clustered into
rectangles (the cited clustering algorithm balances the number of
rectangles against the unflagged cells they cover), and the new level-(l+1)
patches take their values from old level-(l+1) patches where those cover
them, else from level l.  The paper states no formulas; the reading here:

flag     cell of a level-l patch: h > drytol and |h + b - sea_level| > tol;
         then every cell within `buffer` cells (max-norm) of a flagged cell
         of the same patch; then the cells within `margin` cells of the
         patch's edge are cleared (so a new patch and its ghost cells lie over
         the interior of its parent).
cluster  per level-l patch, recursively on a box of its interior (start:
         the whole interior):
         1. shrink the box to the bounding box of its flags (none: no patch);
         2. accept it if flagged / area >= efficiency, or if no side can be
            split (a side can be split when it is at least 2 min_side long);
         3. signatures: flags per column (x) and per row (y) of the box;
            dimensions in order longer side first (ties: x first), only the
            splittable ones; a split at s cuts [lo, hi] into [lo, s] and
            [s + 1, hi], allowed for lo + min_side - 1 <= s <= hi - min_side;
         4. a hole (zero signature) at an allowed s: the one closest to the
            box centre (lo + hi) / 2, ties the smaller s, in the first
            dimension (in order) that has one;
         5. else the strongest inflection over both dimensions: with
            D(k) = sig(k - 1) - 2 sig(k) + sig(k + 1) for lo < k < hi, a
            sign change D(s) D(s + 1) < 0 at an allowed s, strength
            |D(s + 1) - D(s)|; ties: dimension order, then closest to the
            centre, then the smaller s;
         6. else bisect the first dimension: s = (lo + hi) // 2;
         7. cluster both parts.
         A box (in level-l cells) becomes the level-(l+1) patch of r times
         its extent.
fill     new cell (I, J) of level l + 1: the old level-(l+1) patch that
         covers it (first in order) gives its values; otherwise the coarse
         value of oracle/amr.py (linear in space away from the shore, the
         level-l cell under it near the shore) from the one level-l state,
         i.e. with the old and new states equal and alpha = 1.
order    level 2 from level 1, then level 3 from the new level 2, and so on.

Parity unpinned against the paper's code (it cites the clustering algorithm
without stating it); the tests pin the reading by invariants: every flagged
cell is covered, patches of a level do not overlap and lie inside their
parent's interior less the margin, every accepted box meets the efficiency
or cannot be split, the fill copies old cells, reproduces a sea at rest and
interpolates a linear surface exactly.
"""
from __future__ import annotations

import numpy as np

from .amr import OPatch, coarse_value


def flag_patch(q, b, tol, drytol, buffer, margin, sea=0.0):
    """Flags of a patch's interior (my, mx), as the reading above."""
    my, mx = q.shape[0] - 4, q.shape[1] - 4
    base = np.zeros((my, mx), dtype=bool)
    for j in range(my):
        for i in range(mx):
            h = q[j + 2, i + 2, 0]
            if h > drytol and abs(h + b[j + 2, i + 2] - sea) > tol:
                base[j, i] = True
    out = np.zeros_like(base)
    for j in range(my):
        for i in range(mx):
            if base[j, i]:
                out[max(0, j - buffer): j + buffer + 1, max(0, i - buffer): i + buffer + 1] = True
    if margin > 0:
        out[:margin, :] = False
        out[-margin:, :] = False
        out[:, :margin] = False
        out[:, -margin:] = False
    return out


def _allowed(lo, hi, s, min_side):
    return lo + min_side - 1 <= s <= hi - min_side


def cluster(F, efficiency=0.7, min_side=2, box=None):
    """Boxes (i0, j0, i1, j1), inclusive, covering the flags of F[j, i]."""
    my, mx = F.shape
    if box is None:
        box = (0, 0, mx - 1, my - 1)
    i0, j0, i1, j1 = box
    cells = [(i, j) for j in range(j0, j1 + 1) for i in range(i0, i1 + 1) if F[j, i]]
    if not cells:
        return []
    i0 = min(i for i, _ in cells)
    i1 = max(i for i, _ in cells)
    j0 = min(j for _, j in cells)
    j1 = max(j for _, j in cells)
    w, h = i1 - i0 + 1, j1 - j0 + 1
    splittable = {"x": w >= 2 * min_side, "y": h >= 2 * min_side}
    if len(cells) / (w * h) >= efficiency or not (splittable["x"] or splittable["y"]):
        return [(i0, j0, i1, j1)]
    sig = {"x": [sum(1 for j in range(j0, j1 + 1) if F[j, i]) for i in range(i0, i1 + 1)],
           "y": [sum(1 for i in range(i0, i1 + 1) if F[j, i]) for j in range(j0, j1 + 1)]}
    rng = {"x": (i0, i1), "y": (j0, j1)}
    dims = ["x", "y"] if w >= h else ["y", "x"]
    dims = [d for d in dims if splittable[d]]
    split = None
    # holes
    for d in dims:
        lo, hi = rng[d]
        c = (lo + hi) / 2.0
        best = None
        for s in range(lo, hi + 1):
            if sig[d][s - lo] == 0 and _allowed(lo, hi, s, min_side):
                key = (abs(s - c), s)
                if best is None or key < best[0]:
                    best = (key, s)
        if best is not None:
            split = (d, best[1])
            break
    # inflections
    if split is None:
        best = None
        for rank, d in enumerate(dims):
            lo, hi = rng[d]
            c = (lo + hi) / 2.0
            g = sig[d]
            D = {k: g[k - 1 - lo] - 2 * g[k - lo] + g[k + 1 - lo] for k in range(lo + 1, hi)}
            for s in range(lo + 1, hi - 1):
                if D[s] * D[s + 1] < 0 and _allowed(lo, hi, s, min_side):
                    key = (-abs(D[s + 1] - D[s]), rank, abs(s - c), s)
                    if best is None or key < best[0]:
                        best = (key, d, s)
        if best is not None:
            split = (best[1], best[2])
    if split is None:
        d = dims[0]
        lo, hi = rng[d]
        split = (d, (lo + hi) // 2)
    d, s = split
    if d == "x":
        parts = [(i0, j0, s, j1), (s + 1, j0, i1, j1)]
    else:
        parts = [(i0, j0, i1, s), (i0, s + 1, i1, j1)]
    out = []
    for p in parts:
        out += cluster(F, efficiency, min_side, p)
    return out


def new_rects(level_patches, r, tol, drytol, buffer, margin, efficiency=0.7, min_side=2):
    """Level-(l+1) rectangles (i0, j0, mx, my) in the finer level's index from
    the flags of the level-l patches (OPatch objects)."""
    rects = []
    for p in level_patches:
        F = flag_patch(p.q, p.b, tol, drytol, buffer, margin)
        for (a, b_, c, d) in cluster(F, efficiency, min_side):
            gi0, gj0 = p.i0 + a, p.j0 + b_
            rects.append((gi0 * r, gj0 * r, (c - a + 1) * r, (d - b_ + 1) * r))
    return rects


def fill_new(rect, level, H, old_fine, coarse, r, drytol):
    """A new level-(l+1) patch (an OPatch-like object) filled as the reading."""
    i0, j0, mx, my = rect

    class P:  # geometry and state of the new patch
        pass
    p = P()
    p.level, p.i0, p.j0, p.mx, p.my = level, i0, j0, mx, my
    p.b = H.bed_frame(level, i0, j0, mx, my)
    p.q = np.zeros((my + 4, mx + 4, 3))
    for jj in range(my):
        for ii in range(mx):
            I, J = i0 + ii, j0 + jj
            src = next((o for o in old_fine if o.covers(I, J)), None)
            if src is not None:
                p.q[jj + 2, ii + 2] = src.q[src.cell(I, J)]
                continue
            p.q[jj + 2, ii + 2] = coarse_value(coarse, [c.q for c in coarse], r, drytol, 1.0,
                                               I, J, p.b[jj + 2, ii + 2])
    return p


def regrid(hier, H, tol=5e-3, buffer=2, efficiency=0.7, min_side=2, base=1):
    """Regrid every level above level `base` of an oracle Hierarchy in place
    (those levels synchronised with level `base`): level base + 1 from the
    flags of level base, then each finer level from the new level below."""
    from . import BC_USER, grid
    r, P = hier.r, hier.P
    margin = 2 if r == 1 else 1
    for lev in range(base + 1, len(hier.levels) + 1):
        rects = new_rects(hier.levels[lev - 2], r, tol, P.drytol, buffer, margin, efficiency,
                          min_side)
        old = hier.levels[lev - 1]
        new = []
        for rect in rects:
            p = fill_new(rect, lev, H, old, hier.levels[lev - 2], r, P.drytol)
            o = OPatch.__new__(OPatch)
            o.level, o.i0, o.j0, o.mx, o.my = p.level, p.i0, p.j0, p.mx, p.my
            o.q, o.b = p.q, p.b
            o.g = grid(p.mx, p.my, H.dx(lev), H.dx(lev), (BC_USER,) * 4)
            new.append(o)
        hier.levels[lev - 1] = new
    return [[(p.i0, p.j0, p.mx, p.my) for p in lv] for lv in hier.levels]
