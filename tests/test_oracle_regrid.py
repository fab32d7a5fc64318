"""Pins of the reference regridding (oracle/regrid.py): the clustering covers
every flag with disjoint boxes that meet the efficiency or cannot be split,
and handles the textbook cases (one cell, a full block, separated blobs);
flagging marks the disturbed wet cells, the buffer and the cleared margin;
a regridded hierarchy covers every flagged cell, nests inside its parents,
keeps the old values where old patches lie and keeps a sea at rest."""
import numpy as np
import pytest

import oracle as O
from oracle import amr as A
from oracle import regrid as G
from paper_1901_06798_amd import workloads as W


def check_boxes(F, boxes, eff, min_side):
    cov = np.zeros(F.shape, dtype=int)
    for (i0, j0, i1, j1) in boxes:
        assert 0 <= i0 <= i1 < F.shape[1] and 0 <= j0 <= j1 < F.shape[0]
        cov[j0: j1 + 1, i0: i1 + 1] += 1
        sub = F[j0: j1 + 1, i0: i1 + 1]
        w, h = i1 - i0 + 1, j1 - j0 + 1
        assert sub.mean() >= eff or (w < 2 * min_side and h < 2 * min_side)
        # a box is the bounding box of its flags
        assert sub[0, :].any() and sub[-1, :].any() and sub[:, 0].any() and sub[:, -1].any()
    assert cov.max() <= 1
    assert np.all(cov[F] == 1)


def blobs(seed, n=48, k=5):
    rng = np.random.default_rng(seed)
    F = np.zeros((n, n), dtype=bool)
    for _ in range(k):
        cx, cy = rng.integers(0, n, 2)
        rx, ry = rng.integers(1, 8, 2)
        Y, X = np.mgrid[0:n, 0:n]
        F |= ((X - cx) / rx) ** 2 + ((Y - cy) / ry) ** 2 <= 1.0
    F |= rng.random((n, n)) < 0.01
    return F


@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("eff,min_side", [(0.7, 2), (0.85, 3), (0.5, 1)])
def test_clusters_cover_flags_disjointly_and_efficiently(seed, eff, min_side):
    F = blobs(seed)
    check_boxes(F, G.cluster(F, eff, min_side), eff, min_side)


def test_clustering_textbook_cases():
    F = np.zeros((20, 30), dtype=bool)
    assert G.cluster(F) == []
    F[7, 11] = True
    assert G.cluster(F) == [(11, 7, 11, 7)]
    F[:] = False
    F[3:9, 5:17] = True
    assert G.cluster(F) == [(5, 3, 16, 8)]
    # two blocks separated by empty columns: split at a hole, one box each
    F[:] = False
    F[2:10, 1:6] = True
    F[4:12, 20:28] = True
    assert sorted(G.cluster(F)) == [(1, 2, 5, 9), (20, 4, 27, 11)]
    # an L: no hole; the boxes still meet the efficiency
    F[:] = False
    F[2:18, 2:6] = True
    F[14:18, 2:26] = True
    boxes = G.cluster(F, 0.8, 2)
    check_boxes(F, boxes, 0.8, 2)
    assert len(boxes) >= 2


def test_flagging_buffer_and_margin():
    O.lib()
    P = O.params()
    my, mx = 20, 24
    q = np.zeros((my + 4, mx + 4, 3))
    b = np.full((my + 4, mx + 4), -100.0)
    q[..., 0] = 100.0                # sea at rest
    assert not G.flag_patch(q, b, 5e-3, P.drytol, 2, 1).any()
    q[12, 10, 0] = 100.01            # one disturbed cell (interior (10, 8))
    F = G.flag_patch(q, b, 5e-3, P.drytol, 2, 1)
    want = np.zeros((my, mx), dtype=bool)
    want[8:13, 6:11] = True
    assert np.array_equal(F, want)
    q[3, 3, 0] = 100.02              # next to the edge: its buffer is cut by the margin
    F = G.flag_patch(q, b, 5e-3, P.drytol, 2, 1)
    assert not F[0, :].any() and not F[:, 0].any() and F[1, 1] and F[3, 3]
    q[3, 3, 0] = 0.0                 # a dry cell is never flagged
    b[3, 3] = 50.0
    assert not G.flag_patch(q, b, 5e-3, P.drytol, 0, 1)[1, 1]


def test_regridded_hierarchy_covers_flags_and_nests():
    O.lib()
    P = O.params()
    H = W.amr_three_levels(2, bed="shelf", amp=2.0, u0=0.3)
    h = A.Hierarchy(H, P)
    h.run(6.0, 2)
    old2 = [(p.i0, p.j0, p.mx, p.my, p.q.copy()) for p in h.levels[1]]
    rects = G.regrid(h, H, tol=5e-3, buffer=2)
    r = h.r
    assert len(rects[1]) > 0
    for lev in (2, 3):
        parents = h.levels[lev - 2]
        kids = h.levels[lev - 1]
        # every flagged parent cell (with the margin) is covered
        for p in parents:
            F = G.flag_patch(p.q, p.b, 5e-3, P.drytol, 2, 1)
            for j, i in zip(*np.nonzero(F)):
                I, J = (p.i0 + i) * r, (p.j0 + j) * r
                assert any(k.covers(I, J) for k in kids)
        # patches of a level are disjoint; each one with its ghost cells lies
        # over one parent's interior
        for a, k in enumerate(kids):
            for k2 in kids[a + 1:]:
                assert not (k.i0 < k2.i0 + k2.mx and k2.i0 < k.i0 + k.mx
                            and k.j0 < k2.j0 + k2.my and k2.j0 < k.j0 + k.my)
            assert any(p.covers((k.i0 - 2) // r, (k.j0 - 2) // r)
                       and p.covers((k.i0 + k.mx + 1) // r, (k.j0 + k.my + 1) // r)
                       for p in parents)
            assert k.mx % r == 0 and k.my % r == 0
    # cells covered by an old level-2 patch keep its values
    for k in h.levels[1]:
        for (i0, j0, mx, my, q) in old2:
            for J in range(max(k.j0, j0), min(k.j0 + k.my, j0 + my)):
                for I in range(max(k.i0, i0), min(k.i0 + k.mx, i0 + mx)):
                    assert np.array_equal(k.q[k.cell(I, J)], q[J - j0 + 2, I - i0 + 2])
    # the regridded hierarchy runs on
    h.run(6.0, 1)


def test_sea_at_rest_needs_no_refinement_and_fill_keeps_rest():
    O.lib()
    P = O.params()
    H = W.amr_three_levels(4, bed="bowl", amp=0.0)
    h = A.Hierarchy(H, P)
    rects = G.regrid(h, H)
    assert rects[1] == [] and rects[2] == []
    # a patch filled from a level at rest is at rest, bitwise
    h = A.Hierarchy(H, P)
    p = G.fill_new((40, 48, 24, 16), 2, H, [], h.levels[0], 4, P.drytol)
    q = p.q[2:-2, 2:-2]
    assert np.all(q[..., 0] + p.b[2:-2, 2:-2] == 0.0) and not q[..., 1:].any()


def test_new_cells_interpolate_a_linear_surface():
    # a new patch over a tilted sea (all wet, the bowl bed) takes the surface
    # of the level below linearly at its own cell centres, and linear momenta
    O.lib()
    P = O.params()
    r = 4
    H = W.amr_three_levels(r, bed="bowl", amp=0.0)
    h = A.Hierarchy(H, P)
    c = h.levels[0][0]
    dxc, dxf = H.dx(1), H.dx(2)
    n = c.q.shape[0]
    J, I = np.meshgrid(np.arange(n) - 2, np.arange(n) - 2, indexing="ij")
    xc, yc = (I + 0.5) * dxc, (J + 0.5) * dxc
    c.q[..., 0] = (0.3 - 1e-6 * xc + 4e-6 * yc) - c.b
    c.q[..., 1] = 1.0 + 2e-4 * yc
    c.q[..., 2] = -3.0 + 1e-4 * xc
    i0, j0, mx, my = 40, 48, 24, 16
    p = G.fill_new((i0, j0, mx, my), 2, H, [], h.levels[0], r, P.drytol)
    for jj in range(my):
        for ii in range(mx):
            x, y = (i0 + ii + 0.5) * dxf, (j0 + jj + 0.5) * dxf
            qf = p.q[jj + 2, ii + 2]
            assert qf[0] + p.b[jj + 2, ii + 2] == pytest.approx(0.3 - 1e-6 * x + 4e-6 * y,
                                                                 abs=1e-11)
            assert qf[1] == pytest.approx(1.0 + 2e-4 * y, rel=1e-13)
            assert qf[2] == pytest.approx(-3.0 + 1e-4 * x, rel=1e-13)
