"""GPU tests of the heaviest-first launch order (swe_patch_step_sched): the
order is scheduling only, so the states, step sizes and status words equal
those of index-order launches bit for bit; the schedule buffer holds a
permutation of the tasks sorted by the work each recorded, largest first,
ties by index."""
import numpy as np
import pytest

from paper_1901_06798_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1901_06798_amd import _lib as L
    from paper_1901_06798_amd.solver import PatchSolver
    L.lib()
    return L, PatchSolver, torch


def shelf(n):
    # a wave over the deep ocean, water at rest ahead of it and dry land past
    # the shelf: tasks of very different work
    return W.shelf_grid(n, 1000.0, seed=3, sigma=25e3)


# rows per strip task of swe_patch_step (its default), at most the patch's rows
ROWS = 48


def check_schedule(sched, ntask, rows):
    order = sched[:ntask].astype(np.int64)
    cost = sched[ntask:].astype(np.int64)
    assert sorted(order.tolist()) == list(range(1, ntask + 1))
    # a task marches rows + 5 row iterations, each with an x- and a y-sweep
    assert cost.min() >= 0 and cost.max() <= 2 * (rows + 5)
    # bins of `width` units, 16 bins, largest first, ties by task index
    width = (2 * (rows + 5) + 16) // 16
    key = np.minimum(cost // width, 15)
    expect = np.argsort(-key, kind="stable") + 1
    assert np.array_equal(order, expect)
    return cost


@pytest.mark.parametrize("precision,method", [(0, 0), (1, 0), (0, 1)])
def test_ordered_equals_index_order(gpu, precision, method):
    L, PatchSolver, torch = gpu
    pb = shelf(601)
    p = L.params(precision=precision, method=method)
    print(f"case order shelf 601^2 precision={precision} method={method}", flush=True)
    a = PatchSolver(pb, p, ordered=True, order_every=1)
    b = PatchSolver(pb, p, ordered=False)
    ntask = L.swe_patch_tasks(a.pt)
    assert a.sched.numel() == 2 * ntask
    da = a.run(40)
    db = b.run(40)
    torch.cuda.synchronize()
    assert np.array_equal(da, db)
    assert a.cur == b.cur
    assert torch.equal(a.planes(), b.planes())
    assert torch.equal(a.status, b.status)
    assert torch.equal(a.dt, b.dt)
    cost = check_schedule(a.sched.cpu().numpy().view(np.uint32), ntask, ROWS)
    # the tasks differ in work, so the order is not the index order
    assert cost.max() > cost.min()


def test_ordered_device_loop_equals_index_order(gpu):
    L, PatchSolver, torch = gpu
    pb = shelf(480)
    p = L.params()
    print("case order shelf 480^2 device CFL loop", flush=True)
    a = PatchSolver(pb, p, ordered=True)
    b = PatchSolver(pb, p, ordered=False)
    for s in (a, b):
        s.initial_dt()
        s.run_async(60)
    torch.cuda.synchronize()
    assert torch.equal(a.planes(), b.planes())
    assert torch.equal(a.dt, b.dt)
    assert torch.equal(a.status, b.status)


def test_schedule_of_a_small_patch(gpu):
    # fewer tasks than one tile of the sort, a ragged last chunk of rows
    L, PatchSolver, torch = gpu
    pb = W.gaussian_hump(70, 1000.0, sigma=6e3)
    p = L.params()
    a = PatchSolver(pb, p, ordered=True, order_every=1)
    b = PatchSolver(pb, p, ordered=False)
    a.run(12)
    b.run(12)
    torch.cuda.synchronize()
    assert torch.equal(a.planes(), b.planes())
    ntask = L.swe_patch_tasks(a.pt)
    assert ntask == 2 * 2  # 70 columns: 2 strips of 60; 70 rows: 2 chunks of 48
    check_schedule(a.sched.cpu().numpy().view(np.uint32), ntask, ROWS)


@pytest.mark.parametrize("mx,my", [(60, 32), (70, 70), (4096, 4096), (7680, 6144),
                                   (1740, 27120), (8192, 12288)])
def test_order_kernel_is_a_stable_sort(gpu, mx, my):
    # swe_patch_order on recorded work alone (the patch shape sets the task
    # count: 1, 4, 5934, 16384 = one full round of the sort, 16385 and 35072
    # = several rounds)
    L, _, torch = gpu
    pt = L.patch(mx, my, mx + 4, 1.0, 1.0)
    n = L.swe_patch_tasks(pt)
    print(f"case order kernel {mx}x{my} tasks={n}", flush=True)
    rng = np.random.default_rng(n)
    cost = rng.integers(0, 75, n).astype(np.int32)
    cost[: n // 3] = 7  # long runs of equal work
    sched = torch.zeros(2 * n, dtype=torch.int32, device="cuda:0")
    sched[n:] = torch.from_numpy(cost).to("cuda:0")
    sched[:n] = 12345  # stale order: the sort overwrites all of it
    L.swe_patch_order(pt, sched.data_ptr(), sched.numel())
    torch.cuda.synchronize()
    got = sched.cpu().numpy().view(np.uint32)
    assert np.array_equal(got[n:], cost.view(np.uint32))
    check_schedule(got, n, min(ROWS, my))


def test_xcd_runs_give_bitwise_the_same_step(gpu):
    # launch positions dealt to the XCDs in runs of 1, 3 and 8 ranks (the last
    # ranks past a whole block of 8 runs keep their position): any mapping is a
    # permutation of the tasks, so the results are the same bit for bit
    L, PatchSolver, torch = gpu
    pb = shelf(601)
    print("case xcd runs shelf 601^2", flush=True)
    results = []
    for run in (1, 3, 8):
        for ordered in (True, False):
            s = PatchSolver(pb, L.params(), ordered=ordered, launch=L.launch(xcd_run=run))
            dts = s.run(25)
            torch.cuda.synchronize()
            results.append((dts, s.planes().clone(), s.dt.clone()))
    for dts, q, dt in results[1:]:
        assert np.array_equal(dts, results[0][0])
        assert torch.equal(q, results[0][1]) and torch.equal(dt, results[0][2])
