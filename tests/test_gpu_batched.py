"""GPU tests of the batched persistent step: a patch's result is bit for bit
the single-patch result whatever batch, schedule or graph replay it runs in,
and AMR-shaped patch sets (three levels, 1/4/16 substeps) match the reference
solver run patch by patch with the same step sizes."""
import numpy as np
import pytest

from helpers import interior, oracle_setup
from paper_1901_06798_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1901_06798_amd import _lib as L
    from paper_1901_06798_amd.batched import BatchedSolver
    from paper_1901_06798_amd.solver import PatchSolver
    L.lib()
    return L, BatchedSolver, PatchSolver, torch


def mixed_problems():
    from test_gpu_split import smooth_random_problem
    shapes = [(61, 67, (W.BC_EXTRAP,) * 4), (130, 40, (W.BC_WALL,) * 4),
              (17, 19, (W.BC_EXTRAP, W.BC_WALL, W.BC_WALL, W.BC_EXTRAP)),
              (96, 96, (W.BC_EXTRAP,) * 4), (1, 25, (W.BC_EXTRAP, W.BC_EXTRAP, W.BC_WALL, W.BC_WALL)),
              (200, 150, (W.BC_EXTRAP,) * 4)]
    return [smooth_random_problem(mx, my, seed=100 + k, bc=bc) for k, (mx, my, bc) in enumerate(shapes)]


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("seg,rows", [(64, 0), (32, 0), (64, 7), (0, 0), (0, 7)])
def test_batched_equals_single_bitwise(gpu, precision, seg, rows):
    L, BatchedSolver, PatchSolver, torch = gpu
    probs = mixed_problems()
    p = L.params(precision=precision)
    print(f"case batched vs single precision={precision} seg={seg} rows={rows}", flush=True)
    bs = BatchedSolver(probs, p, groups=list(range(len(probs))),
                       sched=L.schedule(seg=seg, rows_per_task=rows))
    bs.initial_dt()
    bs.run(12)
    torch.cuda.synchronize()
    assert bs.flags()[0] & ~L.STATUS_CFL_EXCEEDED == 0
    for k, pb in enumerate(probs):
        s = PatchSolver(pb, p)
        s.initial_dt()
        s.run_async(12)
        torch.cuda.synchronize()
        for a, c in zip(bs.state(k), s.state()):
            assert np.array_equal(a, c), f"patch {k}"


def amr_set(seed=3, counts=(6, 10, 14)):
    specs, probs = W.amr_patch_set(npatch=counts, seed=seed)
    trefs = [s.tref for s in specs]
    return specs, probs, trefs


def test_amr_patch_set_matches_reference(gpu, orc):
    L, BatchedSolver, PatchSolver, torch = gpu
    specs, probs, trefs = amr_set()
    bs = BatchedSolver(probs, L.params(), trefs=trefs)
    bs.initial_dt()
    dts = bs.run(3, record_dt=True)[:, 0]
    torch.cuda.synchronize()
    assert bs.flags() == (0, 0)
    P = orc.params()
    rates = []
    for k, pb in enumerate(probs):
        g, q, b = oracle_setup(orc, pb)
        t = trefs[k]
        for dt in dts:
            orc.run(P, g, q, b, t, dt_forced=[dt / t] * t)
        for f, a in zip(range(3), bs.state(k)):
            ref = interior(q)[..., f]
            scale = max(np.abs(ref).max(), 1e-300)
            assert np.abs(a - ref).max() / scale <= 1e-12, (k, f)
    # the coarse dt follows the CFL rule over all levels (dt_l = dt_1 / tref_l)
    g0 = [oracle_setup(orc, pb) for pb in probs]
    rate = 0.0
    for k, (g, q, b) in enumerate(g0):
        sm = orc.speed_scan(P, g, q, b)
        rate = max(rate, max(sm[0] / g.dx, sm[1] / g.dy) / trefs[k])
    assert dts[0] == pytest.approx(0.9 / rate, rel=1e-15)


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("seg,per_substep", [(32, 0), (64, 1), (32, 1), (0, 1)])
def test_amr_substeps_equal_single_patch_bitwise(gpu, precision, seg, per_substep):
    L, BatchedSolver, PatchSolver, torch = gpu
    specs, probs, trefs = amr_set(seed=5, counts=(3, 4, 5))
    print(f"case AMR substeps precision={precision} seg={seg} per_substep={per_substep}",
          flush=True)
    p = L.params(precision=precision)
    bs = BatchedSolver(probs, p, trefs=trefs,
                       sched=L.schedule(seg=seg, per_substep=per_substep))
    bs.initial_dt()
    dts = bs.run(2, record_dt=True)[:, 0]
    torch.cuda.synchronize()
    for k, pb in enumerate(probs):
        s = PatchSolver(pb, p)
        t = trefs[k]
        sub = []
        for dt in dts:
            sub += [dt / t] * t
        s.run_forced(sub)
        torch.cuda.synchronize()
        for a, c in zip(bs.state(k), s.state()):
            assert np.array_equal(a, c), f"patch {k} tref {t}"


@pytest.mark.parametrize("seg,per_substep", [(64, 0), (64, 1), (0, 1)])
def test_graph_replay_matches_eager(gpu, seg, per_substep):
    L, BatchedSolver, PatchSolver, torch = gpu
    specs, probs, trefs = amr_set(seed=7, counts=(4, 6, 8))
    sched = L.schedule(seg=seg, per_substep=per_substep)
    eager = BatchedSolver(probs, L.params(), trefs=trefs, sched=sched)
    eager.initial_dt()
    graph = BatchedSolver(probs, L.params(), trefs=trefs, sched=sched)
    graph.initial_dt()
    graph.capture(4)
    for rep in range(3):
        eager.run(4)
        graph.replay()
        # the program's own eager work between replays
        x = torch.randn(1000, device=graph.dev).sum()
        torch.cuda.synchronize()
        del x
        for k in range(len(probs)):
            for a, c in zip(eager.state(k), graph.state(k)):
                assert np.array_equal(a, c), f"replay {rep} patch {k}"
    assert graph.flags() == eager.flags()


def test_plan_rejects_user_boundary_with_substeps(gpu):
    L, BatchedSolver, PatchSolver, torch = gpu
    specs, probs, trefs = amr_set(seed=1, counts=(1, 1, 1))
    probs[2].bc = (W.BC_USER,) * 4
    with pytest.raises(L.SweError):
        BatchedSolver(probs, L.params(), trefs=trefs)


@pytest.mark.parametrize("seg", [64, 0])
def test_advance_equals_the_step_by_step_sequence(gpu, seg):
    # swe_batched_advance (one call for n steps with the CFL rule and the
    # retake) against n enqueue_step calls; two groups start above the limit
    L, BatchedSolver, PatchSolver, torch = gpu
    specs, probs, trefs = amr_set(seed=9, counts=(3, 4, 5))
    groups = [k % 4 for k in range(len(probs))]
    sched = L.schedule(seg=seg, per_substep=1 if seg == 0 else 0)
    print(f"case batched advance seg={seg}", flush=True)
    a = BatchedSolver(probs, L.params(), trefs=trefs, groups=groups, sched=sched)
    b = BatchedSolver(probs, L.params(), trefs=trefs, groups=groups, sched=sched)
    for s in (a, b):
        s.initial_dt()
        s.dt.mul_(torch.tensor([1.0, 2.5, 1.0, 1.7], dtype=torch.float64, device=s.dev))
    for _ in range(7):
        a.enqueue_step()
    pending = torch.zeros(2 * b.ngroups, dtype=torch.int32, device=b.dev)
    args = (b.table.data_ptr(), b.n, b.ngroups, b.items.data_ptr(), b.nitems, b.tasks.data_ptr(),
            b.tasks.data_ptr() + L.SWE_TASK_BYTES * (b.ntasks - b.nplain), b.nplain, b.nsub,
            b.pools[0].data_ptr(), b.pools[1].data_ptr(), b.cur,
            b.work.data_ptr() if b.work is not None else 0, 3 * b.plane, b.b.data_ptr(),
            b.dt.data_ptr(), b.smax.data_ptr(), b.status.data_ptr(), 0,
            b.group_flags.data_ptr(), b.retake.data_ptr(), pending.data_ptr(),
            b.queue.data_ptr(), b.sched, 7, b.stream)
    L.swe_batched_advance(b.p, *args)
    b.cur = (b.cur + 7) % 2
    torch.cuda.synchronize()
    assert a.cur == b.cur
    assert int(a.status[0].item()) & L.STATUS_RETAKEN
    # the same flags (no step here resets a depth, so the counts agree too)
    assert torch.equal(a.status, b.status) and torch.equal(a.dt, b.dt)
    assert not pending.any()
    for k in range(len(probs)):
        for x, y in zip(a.state(k), b.state(k)):
            assert np.array_equal(x, y), k


@pytest.mark.parametrize("seg", [64, 32, 0])
def test_fused_cfl_rule_equals_the_separate_launches(gpu, seg):
    # one-launch steps (single-substep patches): swe_batched_advance folds the
    # CFL rule into the step's last workgroup when given the queue words, and
    # launches the rule separately without them; both give the same states,
    # step sizes, flags and per-group conditions bit for bit, and leave the
    # pending pairs and the queue words at zero
    L, BatchedSolver, PatchSolver, torch = gpu
    specs, probs, trefs = amr_set(seed=9, counts=(3, 4, 5))
    groups = [k % 4 for k in range(len(probs))]
    sched = L.schedule(seg=seg)
    print(f"case fused batched CFL rule seg={seg}", flush=True)
    runs = []
    for fused in (True, False):
        s = BatchedSolver(probs, L.params(), trefs=[1] * len(probs), groups=groups, sched=sched)
        assert s.nsub == 1 and (s.nitems == 0) == (seg != 0)
        s.initial_dt()
        s.dt.mul_(torch.tensor([1.0, 2.5, 1.0, 1.7], dtype=torch.float64, device=s.dev))
        pending = torch.zeros(2 * s.ngroups, dtype=torch.int32, device=s.dev)
        gstat = torch.zeros(2 * s.ngroups, dtype=torch.int32, device=s.dev)
        s.queue.zero_()
        for k in range(3):
            L.swe_batched_advance(
                s.p, s.table.data_ptr(), s.n, s.ngroups, s.items.data_ptr(), s.nitems,
                s.tasks.data_ptr(), s.tasks.data_ptr() + L.SWE_TASK_BYTES * (s.ntasks - s.nplain),
                s.nplain, s.nsub, s.pools[0].data_ptr(), s.pools[1].data_ptr(), s.cur, 0,
                3 * s.plane, s.b.data_ptr(), s.dt.data_ptr(), s.smax.data_ptr(),
                s.status.data_ptr(), gstat.data_ptr(), s.group_flags.data_ptr(),
                s.retake.data_ptr(), pending.data_ptr(), s.queue.data_ptr() if fused else 0,
                s.sched, 3, s.stream)
            s.cur = (s.cur + 3) % 2
            if k == 0:
                # a group far above the limit again
                s.dt[3] *= 3.0
        torch.cuda.synchronize()
        assert not pending.any() and not s.queue.any() and not s.smax.any()
        runs.append((s, gstat))
    (a, ga), (b, gb) = runs
    assert int(a.status[0].item()) & L.STATUS_RETAKEN
    assert torch.equal(a.status, b.status) and torch.equal(a.dt, b.dt)
    assert torch.equal(ga, gb) and torch.equal(a.group_flags, b.group_flags)
    for k in range(len(probs)):
        for x, y in zip(a.state(k), b.state(k)):
            assert np.array_equal(x, y), k
