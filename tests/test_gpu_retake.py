"""GPU tests of the CFL rule's retake on the device: a step whose Courant
number exceeds cfl_max is redone, with the reduced step size, by a gated
launch that follows the CFL reduction (no host round trip).  The result is
the reference solver's, which redoes the step on the host, and the host
retake loop's, bit for bit; in a batch only the offending group is redone."""
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
    return L, PatchSolver, BatchedSolver, torch


def too_large_dt(PatchSolver, pb, p, factor):
    s = PatchSolver(pb, p)
    s.initial_dt()
    return float(s.dt.item()) * factor


@pytest.mark.parametrize("precision", [0, 1])
def test_device_retake_equals_host_retake(gpu, orc, precision):
    L, PatchSolver, _, torch = gpu
    pb = W.gaussian_hump(96, 1000.0, sigma=8e3)
    p = L.params(precision=precision)
    big = too_large_dt(PatchSolver, pb, p, 2.2)
    print(f"case retake hump 96x96 precision={precision} dt0={big}", flush=True)
    host = PatchSolver(pb, p)
    host.run(12, dt0=big)
    dev = PatchSolver(pb, p)
    dev.dt.fill_(big)
    dev.run_async(12)
    torch.cuda.synchronize()
    assert host.retakes >= 1
    st = int(dev.status[0].item())
    assert st & L.STATUS_RETAKEN
    assert not st & L.STATUS_CFL_EXCEEDED
    for a, c in zip(host.state(), dev.state()):
        assert np.array_equal(a, c)
    assert float(host.dt.item()) == float(dev.dt.item())
    if precision == 0:
        # and the reference solver, which retakes on the host, agrees exactly
        g, q, b = oracle_setup(orc, pb)
        r = orc.run(orc.params(), g, q, b, 12, dt0=big)
        assert r["retakes"] >= 1
        ref = interior(q)
        for k, a in enumerate(dev.state()):
            assert np.array_equal(a, ref[..., k])


@pytest.mark.parametrize("seg", [64, 0])
def test_batched_retake_redoes_only_the_offending_group(gpu, seg):
    L, PatchSolver, BatchedSolver, torch = gpu
    probs = [W.gaussian_hump(64 + 16 * k, 1000.0, sigma=6e3) for k in range(4)]
    p = L.params()
    factors = [1.0, 2.2, 1.0, 1.6]
    print(f"case batched retake seg={seg}, 4 patches, groups 1 and 3 start above the limit",
          flush=True)
    bs = BatchedSolver(probs, p, groups=list(range(len(probs))), sched=L.schedule(seg=seg))
    bs.initial_dt()
    bs.dt.mul_(torch.tensor(factors, dtype=torch.float64, device=bs.dev))
    bs.run(10)
    torch.cuda.synchronize()
    st = int(bs.status[0].item())
    assert st & L.STATUS_RETAKEN
    assert not st & L.STATUS_CFL_EXCEEDED
    for k, pb in enumerate(probs):
        s = PatchSolver(pb, p)
        s.initial_dt()
        d0 = float(s.dt.item()) * factors[k]
        s.run(10, dt0=d0)
        torch.cuda.synchronize()
        assert (s.retakes >= 1) == (factors[k] > 1.5), f"patch {k}"
        for a, c in zip(bs.state(k), s.state()):
            assert np.array_equal(a, c), f"patch {k}"


def test_retake_flags_are_cleared_each_step(gpu):
    L, PatchSolver, _, torch = gpu
    pb = W.gaussian_hump(64, 1000.0, sigma=6e3)
    p = L.params()
    s = PatchSolver(pb, p)
    s.dt.fill_(too_large_dt(PatchSolver, pb, p, 2.2))
    s.run_async(1)
    torch.cuda.synchronize()
    # the first step was redone, and the redo, within the limit, cleared the flag
    assert int(s.status[0].item()) & L.STATUS_RETAKEN
    assert int(s.retake.item()) == 0
    s.status.zero_()
    s.run_async(1)
    torch.cuda.synchronize()
    # the next one stood: no redo, flag clear
    assert not int(s.status[0].item()) & L.STATUS_RETAKEN
    assert int(s.retake.item()) == 0


@pytest.mark.parametrize("case", ["f64", "f32", "unsplit", "sphere", "f64-large"])
def test_cfl_rule_fused_into_the_step_equals_the_separate_launches(gpu, case):
    # swe_patch_step_cfl + swe_patch_retake_cfl (two launches a step) against
    # the step, swe_cfl_reduce, swe_patch_retake and swe_cfl_reduce (four):
    # the same states, step sizes, flags and status bits, a first step 2.4x
    # the CFL step included; counter and speeds are left at 0
    L, PatchSolver, _, torch = gpu
    if case == "sphere":
        from paper_1901_06798_amd.sphere import SphereSolver as Solver
        pb = W.latlon_basin(130, 90, lat0=40.0, dlon=0.1, dlat=0.1, amp=2.0, sigma_deg=0.7)
        p = L.params()
    elif case == "f64-large":
        # about a hundred waves on every XCD: the last one must see every speed
        Solver = PatchSolver
        pb = W.shelf_grid(1536, 600.0, seed=3, amp=2.0, x_s_frac=0.6, width=30e3)
        p = L.params()
    else:
        Solver = PatchSolver
        pb = W.gaussian_hump(150, 1000.0, sigma=8e3)
    if case in ("f64", "f32", "unsplit"):
        p = L.params(precision=1 if case == "f32" else 0,
                     method=L.UNSPLIT if case == "unsplit" else L.SPLIT)
    print(f"case fused CFL rule {case}", flush=True)
    runs = []
    for fused in (True, False):
        s = Solver(pb, p, order_every=1)
        s.fused = fused
        s.initial_dt()
        s.dt.mul_(2.4)
        dts = []
        for _ in range(12):
            s.enqueue_step()
            dts.append(s.dt.clone())
        torch.cuda.synchronize()
        runs.append((s, torch.stack(dts).cpu().numpy()))
    (a, da), (b, db) = runs
    assert np.array_equal(da, db)
    assert int(a.status[0].item()) & L.STATUS_RETAKEN
    assert torch.equal(a.status, b.status)
    assert not a.counter.any() and not a.smax.any()
    for x, y in zip(a.state(), b.state()):
        assert np.array_equal(x, y)


@pytest.mark.parametrize("rid,n", [(45, 372), (86, 668)])
def test_only_accepted_steps_report_depth_resets(gpu, orc, rid, n):
    # serving scenarios 45 (372^2) and 86 (668^2), 1000 steps: some steps
    # above the Courant limit reset depths before the CFL rule redoes them,
    # and in scenario 86 one redo is still above the limit and is redone
    # again.  The redone steps report nothing: the fused device loop (up to
    # two redos), the host loop and the batched loop (swe_batched_advance, as
    # the server runs it) report no reset, as the reference run does, and end
    # in the reference state bit for bit
    L, PatchSolver, BatchedSolver, torch = gpu
    from paper_1901_06798_amd.serve import Scenario, ScenarioServer
    pb = W.scenario(rid, n=n, nsteps=1000)
    print(f"case scenario {rid} accepted-step conditions", flush=True)
    g, q, b = oracle_setup(orc, pb)
    r = orc.run(orc.params(), g, q, b, 1000)
    assert r["clamps"] == 0 and r["retakes"] > 0
    dev = PatchSolver(pb, L.params())
    dev.initial_dt()
    dev.run_async(1000)
    host = PatchSolver(pb, L.params())
    host.run(1000)
    torch.cuda.synchronize()
    for s in (dev, host):
        f, c = s.flags()
        assert c == 0 and not f & (L.STATUS_NEG_DEPTH | L.STATUS_CFL_EXCEEDED), (f, c)
        for k, a in enumerate(s.state()):
            assert np.array_equal(a, interior(q)[..., k])
    assert dev.flags()[0] & L.STATUS_RETAKEN
    srv = ScenarioServer(L.params(), max_slots=2, steps_per_round=50)
    out = srv.serve([Scenario(rid, 0.0, pb, 1000), Scenario(3, 0.0, W.scenario(3, n=200), 300)])
    assert not out["status_flags"] & L.STATUS_CFL_EXCEEDED
    got = {sc.rid: sc for sc in out["done"]}
    assert got[rid].result["clamps"] == 0 and not got[rid].result["status"] & L.STATUS_NEG_DEPTH
    assert np.array_equal(got[rid].result["eta"], interior(q)[..., 0] + interior(b))
