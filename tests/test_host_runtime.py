"""Host-side pieces of the runtime that need no GPU: the pool allocator of
the scenario server and the batched planner of the C library."""
import os

import pytest

from paper_1901_06798_amd import workloads as W


def test_pool_allocator_first_fit_and_merge():
    from paper_1901_06798_amd.serve import PoolAllocator
    a = PoolAllocator(1000, align=10)
    x = a.alloc(95)
    y = a.alloc(300)
    z = a.alloc(500)
    assert x == (0, 100) and y == (100, 300) and z == (400, 500)
    assert a.alloc(200) is None
    a.release(*y)
    assert a.alloc(250) == (100, 250)
    a.release(100, 250)
    a.release(*x)
    a.release(*z)
    assert a.free == [(0, 1000)]


@pytest.fixture(scope="module")
def L():
    from paper_1901_06798_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_1901_06798_amd import build
        build.build()
    return _lib


def amr_patches(L, counts=(5, 7, 9)):
    specs, probs = W.amr_patch_set(npatch=counts, seed=3)
    pts, off = [], 0
    for s, pb in zip(specs, probs):
        pitch = pb.mx + 4
        size = pitch * (pb.my + 4)
        pts.append(L.patch(pb.mx, pb.my, pitch, pb.dx, pb.dy, off=off, plane_stride=10 ** 8,
                           tref=s.tref, level=s.level, bc=pb.bc))
        off += size
    return specs, pts


@pytest.mark.parametrize("seg", [64, 32])
@pytest.mark.parametrize("per_substep", [0, 1])
def test_plan_covers_every_cell_once(L, seg, per_substep):
    specs, pts = amr_patches(L)
    plan = L.swe_batched_plan(pts, L.schedule(seg=seg, per_substep=per_substep))
    items, ni, tasks, nt, npl = plan.items, plan.nitems, plan.tasks, plan.ntasks, plan.nplain
    cover = {}
    for k in range(nt):
        t = tasks[k]
        p = pts[t.patch]
        c0 = t.strip * (seg - 4) + 2
        assert t.col0 == t.strip * (seg - 4) and t.lanes == seg
        for r in range(t.row0, t.row0 + t.rows):
            for c in range(c0, min(c0 + seg - 4, p.mx + 2)):
                cover[(t.patch, r, c)] = cover.get((t.patch, r, c), 0) + 1
    expect = sum(p.mx * p.my for p in pts)
    assert len(cover) == expect and set(cover.values()) == {1}
    # a patch with substeps is one item holding all its tasks (or, launched
    # per substep, plain like the rest); the plain tasks are the last npl
    # tasks, in no item, ordered by tref, largest first
    seen = []
    for i in range(ni):
        it = items[i]
        assert pts[it.patch].tref > 1 and it.substeps == pts[it.patch].tref
        assert all(tasks[k].patch == it.patch for k in range(it.task_begin, it.task_end))
        seen += list(range(it.task_begin, it.task_end))
    assert sorted(seen) == list(range(nt - npl))
    plain_patches = {tasks[k].patch for k in range(nt - npl, nt)}
    if per_substep:
        assert ni == 0 and npl == nt and plain_patches == set(range(len(pts)))
        assert plan.nsub == max(p.tref for p in pts)
    else:
        assert plain_patches == {k for k, p in enumerate(pts) if p.tref == 1}
        assert plan.nsub == 1
    trefs = [pts[tasks[k].patch].tref for k in range(nt - npl, nt)]
    assert trefs == sorted(trefs, reverse=True)
    # plain tasks are at most 32 rows by default
    assert all(tasks[k].rows <= 32 for k in range(nt - npl, nt))


@pytest.mark.parametrize("rows", [0, 7, 32, 96])
def test_packed_plan_covers_every_cell_once(L, rows):
    # seg = 0: packs of side-by-side segments; every interior cell of every
    # patch is updated by exactly one task, packs hold at most 64 lanes and
    # one tref, and runs are laid tallest first within a tref
    specs, pts = amr_patches(L, (9, 23, 41))
    plan = L.swe_batched_plan(pts, L.schedule(seg=0, rows_per_task=rows))
    items, ni, tasks, nt, npl = plan.items, plan.nitems, plan.tasks, plan.ntasks, plan.nplain
    assert npl == nt and ni > 0 and plan.nsub == max(p.tref for p in pts)
    cover = {}
    H = rows or 48
    prev_tref, prev_rows = None, None
    for i in range(ni):
        it = items[i]
        assert it.patch == -1 and it.task_end > it.task_begin
        if i > 0:
            assert it.task_begin == items[i - 1].task_end
        assert sum(tasks[k].lanes for k in range(it.task_begin, it.task_end)) <= 64
        for k in range(it.task_begin, it.task_end):
            t = tasks[k]
            p = pts[t.patch]
            assert p.tref == it.substeps
            assert 5 <= t.lanes <= 64 and 0 <= t.col0 and t.col0 + t.lanes - 4 <= p.mx
            assert 1 <= t.rows <= H and 2 <= t.row0 and t.row0 + t.rows <= p.my + 2
            # runs of one patch differ by at most one row
            assert t.rows in (-(-p.my // -(-p.my // H)), p.my // -(-p.my // H))
            if prev_tref is not None:
                assert (p.tref, t.rows) <= (prev_tref, prev_rows) or p.tref < prev_tref
            prev_tref, prev_rows = p.tref, t.rows
            # a cut leaves at least 4 columns unless the patch is narrower
            assert t.lanes - 4 >= min(4, p.mx)
            for r in range(t.row0, t.row0 + t.rows):
                for c in range(t.col0 + 2, t.col0 + t.lanes - 2):
                    cover[(t.patch, r, c)] = cover.get((t.patch, r, c), 0) + 1
    assert items[ni - 1].task_end == nt
    assert len(cover) == sum(p.mx * p.my for p in pts) and set(cover.values()) == {1}
    # the packs use most of their lanes
    used = sum(tasks[k].lanes for k in range(nt))
    assert used / (64 * ni) > 0.85


def test_plan_orders_longest_first(L):
    specs, pts = amr_patches(L)
    plan = L.swe_batched_plan(pts, L.schedule(order=0))
    items, ni, tasks = plan.items, plan.nitems, plan.tasks

    def cost(it):
        p = pts[it.patch]
        return sum((tasks[k].rows + 4) for k in range(it.task_begin, it.task_end)) * it.substeps
    costs = [cost(items[i]) for i in range(ni)]
    assert costs == sorted(costs, reverse=True)


def test_plan_rejects_bad_input(L):
    specs, pts = amr_patches(L, (1, 1, 1))
    bad = L.schedule(seg=48)
    with pytest.raises(L.SweError):
        L.swe_batched_plan(pts, bad)
    pts[2].bc[0] = L.BC_USER
    with pytest.raises(L.SweError, match="tref"):
        L.swe_batched_plan(pts, L.schedule())
