"""Pins of the reference AMR level coupling (oracle/amr.py): a sea at rest
stays bitwise at rest across levels; with refinement ratio 1 the hierarchy
reproduces the single-level run cell for cell; averaging takes a linear
surface and linear momenta to the coarse cell-centre values; away from the
shore the ghost fill interpolates linearly in space (bilinear functions,
every cell different, are reproduced at the fine cell centres, over a flat
and over a varying bed) and in time, takes the same level's cell where one
exists, and falls back to the cell under the ghost where a stencil cell is
dry or outside the level below."""
import numpy as np
import pytest

import oracle as O
from oracle import amr as A
from paper_1901_06798_amd import workloads as W


@pytest.fixture(scope="module")
def P():
    O.lib()
    return O.params()


@pytest.mark.parametrize("ratio", [2, 4])
def test_sea_at_rest_stays_bitwise_at_rest(P, ratio):
    H = W.amr_three_levels(ratio, bed="bowl", amp=0.0)
    h = A.Hierarchy(H, P)
    h.run(15.0, 2)
    for lev in (1, 2, 3):
        for p in h.levels[lev - 1]:
            q = p.q[2:-2, 2:-2]
            assert np.all(q[..., 1] == 0.0) and np.all(q[..., 2] == 0.0)
            assert np.all(q[..., 0] + p.b[2:-2, 2:-2] == 0.0)


def single_level(H, P, dt, n):
    p = [x for x in H.patches if x.level == 1][0]
    g = O.grid(p.mx, p.my, H.dx1, H.dx1, H.bc)
    q, b = O.new_state(p.h, p.hu, p.hv, p.b_frame[2:-2, 2:-2])
    O.ghost_fill_b(g, b)
    for _ in range(n):
        O.ghost_fill(g, q)
        out, _, _, nf = O.step(P, g, q, b, dt)
        assert nf == 0
        q[2:-2, 2:-2] = out[2:-2, 2:-2]
    return q


def test_ratio_one_reproduces_the_single_level_run(P):
    # a moving hump over the shelf: every level covers cells of the same
    # size, so fine patches are windows of the coarse grid; the values agree
    # up to the rounding of (h + b) - b in the fill and the average
    H = W.amr_three_levels(1, bed="shelf", amp=2.0, u0=0.3)
    h = A.Hierarchy(H, P)
    dt, n = 60.0, 6
    h.run(dt, n)
    ref = single_level(H, P, dt, n)
    scale = np.abs(ref[2:-2, 2:-2]).max(axis=(0, 1))
    for lev in (1, 2, 3):
        for p in h.levels[lev - 1]:
            r0, c0 = p.j0 + 2, p.i0 + 2
            want = ref[r0: r0 + p.my, c0: c0 + p.mx]
            got = p.q[2:-2, 2:-2]
            err = (np.abs(got - want).max(axis=(0, 1)) / scale).max()
            assert err <= 1e-12, (lev, err)
    # and the run moved water: not a trivially static state
    assert np.abs(ref[2:-2, 2:-2, 1]).max() > 1.0


def test_average_of_linear_fields_is_the_centre_value(P):
    r = 4
    H = W.amr_three_levels(r, bed="flat", amp=0.0)
    h = A.Hierarchy(H, P)
    f = h.levels[1][0]
    dxf = H.dx(2)
    xs = (np.arange(f.mx) + f.i0 + 0.5) * dxf
    ys = (np.arange(f.my) + f.j0 + 0.5) * dxf
    X, Y = np.meshgrid(xs, ys)
    eta = 0.25 + 1e-5 * X - 2e-5 * Y
    f.q[2:-2, 2:-2, 0] = eta - f.b[2:-2, 2:-2]
    f.q[2:-2, 2:-2, 1] = 3.0 + 1e-4 * X
    f.q[2:-2, 2:-2, 2] = -1.0 + 2e-4 * Y
    h.average(1)
    c = h.levels[0][0]
    dxc = H.dx(1)
    for Jc in range(f.j0 // r, (f.j0 + f.my) // r):
        for Ic in range(f.i0 // r, (f.i0 + f.mx) // r):
            xc, yc = (Ic + 0.5) * dxc, (Jc + 0.5) * dxc
            rc, cc = c.cell(Ic, Jc)
            assert c.q[rc, cc, 0] + c.b[rc, cc] == pytest.approx(0.25 + 1e-5 * xc - 2e-5 * yc,
                                                                abs=1e-10)
            assert c.q[rc, cc, 1] == pytest.approx(3.0 + 1e-4 * xc, rel=1e-13)
            assert c.q[rc, cc, 2] == pytest.approx(-1.0 + 2e-4 * yc, rel=1e-12)


def stencil_inside(c, X, Y):
    """True when the bilinear stencil of the point (X, Y), in coarse cell
    units, lies in the interior of the coarse patch c."""
    i0, j0 = int(np.floor(X)), int(np.floor(Y))
    i1 = i0 + (1 if X > i0 else 0)
    j1 = j0 + (1 if Y > j0 else 0)
    return all(c.covers(i, j) for i in (i0, i1) for j in (j0, j1))


@pytest.mark.parametrize("r", [2, 4])
def test_fill_interpolates_bilinear_fields_in_space_and_time(P, r):
    H = W.amr_three_levels(r, bed="flat", amp=0.0)
    h = A.Hierarchy(H, P)
    c = h.levels[0][0]
    n = c.q.shape[0]
    # every coarse cell different: depth 1000 + I + 100 J, momenta I - J and
    # I J (bilinear functions, which bilinear interpolation reproduces)
    J, I = np.meshgrid(np.arange(n) - 2, np.arange(n) - 2, indexing="ij")
    old = [c.q.copy()]
    old[0][..., 0] = 1000.0 + I + 100.0 * J
    old[0][..., 1] = I - J
    old[0][..., 2] = I * J
    c.q[..., 0] = 2000.0 + I + 100.0 * J
    c.q[..., 1] = 2.0 * (I - J)
    c.q[..., 2] = 3.0 * I * J
    checked = {"linear": 0, "constant": 0}
    for alpha in (0.0, 0.5, 0.75):
        h.fill(2, old, alpha)
        for f in h.levels[1]:
            other = [s for s in h.levels[1] if s is not f][0]
            for row in range(f.my + 4):
                for col in range(f.mx + 4):
                    if 2 <= row < f.my + 2 and 2 <= col < f.mx + 2:
                        continue
                    If, Jf = f.i0 + col - 2, f.j0 + row - 2
                    if other.covers(If, Jf):
                        assert np.array_equal(f.q[row, col], other.q[other.cell(If, Jf)])
                        continue
                    X, Y = (If + 0.5) / r - 0.5, (Jf + 0.5) / r - 0.5
                    if not stencil_inside(c, X, Y):
                        X, Y = If // r, Jf // r
                        checked["constant"] += 1
                    else:
                        checked["linear"] += 1
                    want = ((1 - alpha) * (1000.0 + X + 100.0 * Y)
                            + alpha * (2000.0 + X + 100.0 * Y),
                            (1 - alpha) * (X - Y) + alpha * 2.0 * (X - Y),
                            (1 - alpha) * (X * Y) + alpha * 3.0 * X * Y)
                    assert f.q[row, col] == pytest.approx(want, rel=1e-13, abs=1e-12)
    assert checked["linear"] > 100


def test_fill_reproduces_a_linear_surface_over_a_varying_bed(P):
    # the surface, not the depth, is interpolated: a tilted surface over the
    # bowl bed (all wet) comes out tilted at the fine cell centres, whatever
    # the fine cells' own bed; momenta linear in x and y likewise
    r = 4
    H = W.amr_three_levels(r, bed="bowl", amp=0.0)
    h = A.Hierarchy(H, P)
    c = h.levels[0][0]
    dxc = H.dx(1)
    n = c.q.shape[0]
    J, I = np.meshgrid(np.arange(n) - 2, np.arange(n) - 2, indexing="ij")
    xc, yc = (I + 0.5) * dxc, (J + 0.5) * dxc
    eta = 0.4 + 2e-6 * xc - 3e-6 * yc
    c.q[..., 0] = eta - c.b
    c.q[..., 1] = 5.0 + 1e-4 * xc
    c.q[..., 2] = -2.0 + 3e-4 * yc
    h.fill(2, [c.q.copy()], 1.0)
    dxf = H.dx(2)
    nlin = 0
    for f in h.levels[1]:
        other = [s for s in h.levels[1] if s is not f][0]
        for row in range(f.my + 4):
            for col in range(f.mx + 4):
                if 2 <= row < f.my + 2 and 2 <= col < f.mx + 2:
                    continue
                If, Jf = f.i0 + col - 2, f.j0 + row - 2
                X, Y = (If + 0.5) / r - 0.5, (Jf + 0.5) / r - 0.5
                if other.covers(If, Jf) or not stencil_inside(c, X, Y):
                    continue
                x, y = (If + 0.5) * dxf, (Jf + 0.5) * dxf
                assert f.q[row, col, 0] + f.b[row, col] == pytest.approx(
                    0.4 + 2e-6 * x - 3e-6 * y, abs=1e-11)
                assert f.q[row, col, 1] == pytest.approx(5.0 + 1e-4 * x, rel=1e-13)
                assert f.q[row, col, 2] == pytest.approx(-2.0 + 3e-4 * y, rel=1e-13)
                nlin += 1
    assert nlin > 100


def test_dry_stencil_cell_falls_back_to_the_cell_under_the_ghost(P):
    # near the shore (a dry cell in the bilinear stencil, in either state)
    # the ghost takes the coarse cell under it, constant in space
    r = 2
    H = W.amr_three_levels(r, bed="flat", amp=0.0)
    h = A.Hierarchy(H, P)
    c = h.levels[0][0]
    n = c.q.shape[0]
    J, I = np.meshgrid(np.arange(n) - 2, np.arange(n) - 2, indexing="ij")
    c.q[..., 0] = 1000.0 + I + 100.0 * J
    c.q[..., 1] = 0.0
    c.q[..., 2] = 0.0
    f = h.levels[1][0]
    # the coarse cell left of the patch's first interior column, at its first row
    Ic, Jc = f.i0 // r - 1, f.j0 // r
    old = c.q.copy()
    old[c.cell(Ic, Jc)] = 0.0  # dry before the step only
    h.fill(2, [old], 0.5)
    hit = 0
    for row in range(f.my + 4):
        for col in range(f.mx + 4):
            if 2 <= row < f.my + 2 and 2 <= col < f.mx + 2:
                continue
            If, Jf = f.i0 + col - 2, f.j0 + row - 2
            X, Y = (If + 0.5) / r - 0.5, (Jf + 0.5) / r - 0.5
            i0, j0 = int(np.floor(X)), int(np.floor(Y))
            if not (i0 <= Ic <= i0 + 1 and j0 <= Jc <= j0 + 1):
                continue
            under = c.cell(If // r, Jf // r)
            want_eta = 0.5 * (old[under][0] + c.b[under]) + 0.5 * (c.q[under][0] + c.b[under])
            if old[under][0] <= P.drytol and c.q[under][0] <= P.drytol:
                want_eta = f.b[row, col]
            assert f.q[row, col, 0] == max(want_eta - f.b[row, col], 0.0)
            hit += 1
    assert hit >= 4


def test_fill_and_average_keep_dry_land_dry(P):
    # a fully dry level below gives dry ghosts; fully dry fine cells average
    # to a dry coarse cell
    r = 2
    H = W.amr_three_levels(r, bed="flat", amp=0.0)
    h = A.Hierarchy(H, P)
    c = h.levels[0][0]
    c.q[...] = 0.0
    h.fill(2, [c.q.copy()], 0.5)
    for f in h.levels[1]:
        other = [s for s in h.levels[1] if s is not f][0]
        for row in range(f.my + 4):
            for col in range(f.mx + 4):
                inner = 2 <= row < f.my + 2 and 2 <= col < f.mx + 2
                if not inner and not other.covers(f.i0 + col - 2, f.j0 + row - 2):
                    assert np.all(f.q[row, col] == 0.0)
    for s in h.levels[1]:
        s.q[...] = 0.0
    c.q[...] = 7.0
    h.average(1)
    for s in h.levels[1]:
        for Jc in range(s.j0 // r, (s.j0 + s.my) // r):
            for Ic in range(s.i0 // r, (s.i0 + s.mx) // r):
                assert np.all(c.q[c.cell(Ic, Jc)] == 0.0)


def test_cfl_step_of_a_sea_at_rest_is_the_closed_form(P):
    # every level of a flat sea at rest has the same rate sqrt(g H) / dx_1
    # (dx_l = dx_1 / r^(l-1), divided by r^(l-1)): dt_1 = 0.9 dx_1 / sqrt(g H)
    for r in (2, 4):
        H = W.amr_three_levels(r, bed="flat", amp=0.0)
        h = A.Hierarchy(H, P)
        dts, retakes = h.integrate(3)
        want = 0.9 * H.dx1 / np.sqrt(9.81 * H.depth)
        assert retakes == 0
        assert np.allclose(dts, want, rtol=1e-14, atol=0)


@pytest.mark.parametrize("ratio", [2, 4])
def test_cfl_steps_keep_the_courant_number(P, ratio):
    H = W.amr_three_levels(ratio, bed="shelf", amp=2.0, u0=0.3)
    h = A.Hierarchy(H, P)
    dts, retakes = h.integrate(4)
    assert retakes == 0 and len(dts) == 4
    # every accepted step had its rate at most cfl_max / dt
    h2 = A.Hierarchy(H, P)
    d = h2.initial_dt()
    assert dts[0] == d
    for k in range(4):
        h2.reset_speeds()
        h2.advance(1, dts[k])
        rate = h2.rate()
        assert dts[k] * rate <= P.cfl_max
        if k + 1 < 4:
            assert dts[k + 1] == P.cfl_desired / rate


def test_a_coarse_step_above_the_limit_is_redone_from_the_snapshot(P):
    H = W.amr_three_levels(2, bed="shelf", amp=2.0, u0=0.3)
    h = A.Hierarchy(H, P)
    dts, retakes = h.integrate(3, dt0=40.0)  # far above the CFL limit
    assert retakes == 1 and dts[0] < 40.0
    # the retaken run is the run started with the retake's step size
    h2 = A.Hierarchy(H, P)
    dts2, retakes2 = h2.integrate(3, dt0=dts[0])
    assert retakes2 == 0 and np.array_equal(dts, dts2)
    for lev in range(3):
        for p, q in zip(h.levels[lev], h2.levels[lev]):
            assert np.array_equal(p.q, q.q)


def test_regrid_every_b_steps_of_each_level(P):
    # level l + 1 and finer are regridded at the start of every b-th step of
    # level l: with r = 2, b = 2, three coarse steps, level 1 steps 0..2 and
    # level 2 steps 0..5 (two per coarse step)
    H = W.amr_three_levels(2, bed="shelf", amp=2.0, u0=0.3)
    h = A.Hierarchy(H, P)
    h.integrate(3, regrid_every=2)
    assert h.regrids == [(2, 2), (1, 2), (2, 4)]
    # the regridded hierarchy still nests: every level-3 patch and its ghost
    # frame lie over level-2 interiors, every level-2 patch over level 1
    for lev in (2, 3):
        for f in h.levels[lev - 1]:
            for J in range(f.j0 - 2, f.j0 + f.my + 2):
                for I in range(f.i0 - 2, f.i0 + f.mx + 2):
                    assert any(c.covers(I // 2, J // 2) for c in h.levels[lev - 2])


class Cellwise(A.Hierarchy):
    """The hierarchy with the fill and the average taken one cell at a time."""

    def fill(self, lev, old, alpha):
        self.fill_cellwise(lev, old, alpha)

    def average(self, lev):
        self.average_cellwise(lev)


def same_bits(a, b):
    return np.array_equal(a, b) and np.array_equal(np.signbit(a), np.signbit(b))


@pytest.mark.parametrize("kind,ratio", [("three", 1), ("three", 2), ("nested", 2),
                                        ("nested", 4)])
def test_whole_patch_fill_and_average_equal_the_cellwise_rule(P, kind, ratio):
    # the array forms of fill and average against the reading written out
    # cell by cell, bit for bit, over coarse steps of a moving hump; in the
    # small nested hierarchy the finer levels reach over the dry coast, so
    # ghost cells over dry land, the shoreline fallback, copies from the same
    # level and bilinear interpolation all occur
    if kind == "three":
        H = W.amr_three_levels(ratio, bed="shelf", amp=3.0, u0=0.4)
        dt = 8.0
    else:
        H = W.amr_nested(n1=64, ratio=ratio, counts=(3, 4), sizes=(4 * ratio, 8 * ratio),
                         amp=3.0)
        dt = 20.0
    a, b = A.Hierarchy(H, P), Cellwise(H, P)
    for h in (a, b):
        h.run(dt, 2 if ratio == 4 else 3)
    for lev in (1, 2, 3):
        for pa, pb in zip(a.levels[lev - 1], b.levels[lev - 1]):
            assert same_bits(pa.q, pb.q), lev
    if kind == "nested":
        for lev in (2, 3):
            assert any((p.q[..., 0] <= P.drytol).any() for p in a.levels[lev - 1])
            assert any((p.q[2:-2, 2:-2, 0] > 1.0).any() for p in a.levels[lev - 1])
