"""GPU tests of the AMR level coupling (swe_amr_fill, swe_amr_average and the
recursive level stepping of amr.AmrSolver) against the reference hierarchy
(oracle/amr.py): every patch of every level after several coarse steps, to
the FP64 bar (relative 1e-12 per field); a sea at rest stays bitwise at rest;
a captured coarse step replays to the eager result."""
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
    from paper_1901_06798_amd.amr import AmrSolver
    L.lib()
    return L, AmrSolver, torch


def run_oracle(H, dt1, n):
    import oracle as O
    from oracle import amr as A
    O.lib()
    h = A.Hierarchy(H, O.params())
    h.run(dt1, n)
    return h


@pytest.mark.parametrize("ratio,ncoarse", [(1, 4), (2, 3), (4, 2)])
def test_hierarchy_matches_the_reference(gpu, ratio, ncoarse):
    L, AmrSolver, torch = gpu
    H = W.amr_three_levels(ratio, bed="shelf", amp=2.0, u0=0.3)
    dt1 = 6.0
    print(f"case amr three levels ratio={ratio} coarse steps={ncoarse}", flush=True)
    s = AmrSolver(H, L.params())
    s.set_dt(dt1)
    s.run(ncoarse)
    torch.cuda.synchronize()
    ref = run_oracle(H, dt1, ncoarse)
    assert s.flags() == (0, 0)
    assert s.courant() < 1.0
    for lev in range(1, 4):
        pats = ref.levels[lev - 1]
        scale = [max(np.abs(p.q[2:-2, 2:-2, c]).max() for p in pats) for c in range(3)]
        for k, p in enumerate(pats):
            got = s.state(lev, k)
            for c in range(3):
                want = p.q[2:-2, 2:-2, c]
                err = np.abs(got[c] - want).max() / max(scale[c], 1e-300)
                assert err <= 1e-12, (lev, k, c, err)
    # the hierarchy did move water at every level
    assert all(np.abs(s.state(lev, 0)[1]).max() > 0.1 for lev in (1, 2, 3))


def test_sea_at_rest_stays_bitwise_at_rest(gpu):
    L, AmrSolver, torch = gpu
    H = W.amr_three_levels(4, bed="bowl", amp=0.0)
    s = AmrSolver(H, L.params())
    s.set_dt(5.0)
    s.run(2)
    torch.cuda.synchronize()
    for lev in range(1, 4):
        for k, p in enumerate([q for q in H.patches if q.level == lev]):
            h, hu, hv = s.state(lev, k)
            assert np.all(hu == 0.0) and np.all(hv == 0.0)
            assert np.all(h + p.b_frame[2:-2, 2:-2] == 0.0)


def test_captured_coarse_steps_replay_to_the_eager_result(gpu):
    L, AmrSolver, torch = gpu
    H = W.amr_three_levels(2, bed="shelf", amp=2.0, u0=0.3)
    eager = AmrSolver(H, L.params())
    eager.set_dt(6.0)
    eager.run(6)
    g = AmrSolver(H, L.params())
    g.set_dt(6.0)
    g.capture(2)
    for _ in range(3):
        g.replay()
        torch.cuda.synchronize()
        _ = torch.zeros(16, device="cuda:0").sum().item()  # eager work between replays
    torch.cuda.synchronize()
    for lev in range(1, 4):
        for k in range(len([p for p in H.patches if p.level == lev])):
            a = eager.state(lev, k)
            b = g.state(lev, k)
            for c in range(3):
                assert np.array_equal(a[c], b[c]), (lev, k, c)


def rounded_to_fp32(H):
    """The hierarchy as the FP32 surface-deviation path stores it: bed and
    surface deviation rounded to FP32 (sea level 0), depth from them."""
    import copy
    R = copy.deepcopy(H)
    for p in R.patches:
        b64 = p.b_frame
        b32 = b64.astype(np.float32).astype(np.float64)
        inner = b64[2:-2, 2:-2]
        eta = np.where(p.h > 0.0, p.h + inner, inner).astype(np.float32).astype(np.float64)
        p.b_frame = b32
        p.h = np.where(p.h > 0.0, np.maximum(eta - b32[2:-2, 2:-2], 0.0), 0.0)
        p.hu = p.hu.astype(np.float32).astype(np.float64)
        p.hv = p.hv.astype(np.float32).astype(np.float64)
    return R


@pytest.mark.parametrize("ratio", [2, 4])
def test_fp32_deviation_hierarchy_within_1e5_m(gpu, ratio):
    L, AmrSolver, torch = gpu
    H = W.amr_three_levels(ratio, bed="shelf", amp=2.0, u0=0.3)
    print(f"case amr three levels fp32 deviation ratio={ratio}", flush=True)
    s = AmrSolver(H, L.params(precision=L.F32_DEV))
    s.set_dt(6.0)
    s.run(3)
    torch.cuda.synchronize()
    ref = run_oracle(rounded_to_fp32(H), 6.0, 3)
    assert s.flags() == (0, 0)
    worst = 0.0
    for lev in range(1, 4):
        pats = ref.levels[lev - 1]
        mom = max(np.abs(p.q[2:-2, 2:-2, 1]).max() for p in pats)
        for k, p in enumerate(pats):
            h, hu, hv = s.state(lev, k)
            b = p.b[2:-2, 2:-2]
            want = p.q[2:-2, 2:-2]
            wet = (want[..., 0] > 1e-2) & (h > 1e-2)
            err = np.abs((h + b) - (want[..., 0] + b))[wet].max() if wet.any() else 0.0
            worst = max(worst, err)
            assert err <= 1e-5, (lev, k, err)
            assert np.abs(hu - want[..., 1]).max() <= 1e-4 * mom, (lev, k)
    print(f"fp32 deviation hierarchy: max surface difference {worst:.3e} m", flush=True)


def compare_hierarchies(s, ref, tol=1e-12):
    assert s.nlev == len([lv for lv in ref.levels if lv]) or s.nlev == len(ref.levels)
    for lev in range(1, s.nlev + 1):
        pats = ref.levels[lev - 1]
        assert [(p.i0, p.j0, p.mx, p.my) for p in s.lpatches[lev - 1]] == \
            [(p.i0, p.j0, p.mx, p.my) for p in pats], lev
        scale = [max(np.abs(p.q[2:-2, 2:-2, c]).max() for p in pats) for c in range(3)]
        for k, p in enumerate(pats):
            got = s.state(lev, k)
            for c in range(3):
                err = np.abs(got[c] - p.q[2:-2, 2:-2, c]).max() / max(scale[c], 1e-300)
                assert err <= tol, (lev, k, c, err)


@pytest.mark.parametrize("ratio", [2, 4])
def test_cfl_integration_matches_the_reference(gpu, ratio):
    # dt_1 from the CFL condition over every level, on the device after each
    # coarse step, against the reference hierarchy's integration
    L, AmrSolver, torch = gpu
    from oracle import amr as A
    import oracle as O
    H = W.amr_three_levels(ratio, bed="shelf", amp=2.0, u0=0.3)
    print(f"case amr cfl integration ratio={ratio}", flush=True)
    s = AmrSolver(H, L.params())
    dts, rt = s.integrate(4)
    torch.cuda.synchronize()
    O.lib()
    ref = A.Hierarchy(H, O.params())
    rdts, rrt = ref.integrate(4)
    assert rt == rrt == 0
    np.testing.assert_allclose(dts, rdts, rtol=1e-13, atol=0)
    assert s.flags() == (0, 0)
    compare_hierarchies(s, ref)


def test_cfl_retake_of_a_coarse_step(gpu):
    L, AmrSolver, torch = gpu
    from oracle import amr as A
    import oracle as O
    H = W.amr_three_levels(2, bed="shelf", amp=2.0, u0=0.3)
    print("case amr retake from dt0 = 40 s", flush=True)
    s = AmrSolver(H, L.params())
    dts, rt = s.integrate(3, dt0=40.0)
    O.lib()
    ref = A.Hierarchy(H, O.params())
    rdts, rrt = ref.integrate(3, dt0=40.0)
    assert rt == rrt == 1
    np.testing.assert_allclose(dts, rdts, rtol=1e-13, atol=0)
    compare_hierarchies(s, ref)


@pytest.mark.parametrize("ratio", [2, 4])
def test_regrid_every_b_steps_inside_the_integration(gpu, ratio):
    L, AmrSolver, torch = gpu
    from oracle import amr as A
    import oracle as O
    H = W.amr_three_levels(ratio, bed="shelf", amp=2.0, u0=0.3)
    print(f"case amr regrid every 2 level steps ratio={ratio}", flush=True)
    s = AmrSolver(H, L.params())
    dts, rt = s.integrate(3, regrid_every=2)
    O.lib()
    ref = A.Hierarchy(H, O.params())
    rdts, rrt = ref.integrate(3, regrid_every=2)
    assert s.regrids == ref.regrids and len(s.regrids) >= 2
    np.testing.assert_allclose(dts, rdts, rtol=1e-13, atol=0)
    compare_hierarchies(s, ref)


@pytest.mark.parametrize("precision", [0, 1])
def test_bench_hierarchy_matches_the_reference(gpu, precision):
    # the benchmark's hierarchy at its full size (one 1024^2 level-1 patch,
    # 64 level-2 and 128 level-3 patches of 96-160 cells, ratio 4, over the
    # shelf break and the dry coast): two coarse steps of 8 s against the
    # reference hierarchy, every patch of every level; FP64 to 1e-12 per
    # field, the FP32 deviation path within 1e-5 m on cells wet in both
    L, AmrSolver, torch = gpu
    H = W.amr_nested()
    print(f"case amr bench hierarchy precision={precision}", flush=True)
    s = AmrSolver(H, L.params(precision=precision))
    s.set_dt(8.0)
    s.run(2)
    torch.cuda.synchronize()
    assert s.flags() == (0, 0)
    if precision == 0:
        ref = run_oracle(H, 8.0, 2)
        compare_hierarchies(s, ref)
        return
    ref = run_oracle(rounded_to_fp32(H), 8.0, 2)
    worst = 0.0
    for lev in range(1, 4):
        for k, p in enumerate(ref.levels[lev - 1]):
            h, hu, hv = s.state(lev, k)
            b = p.b[2:-2, 2:-2]
            want = p.q[2:-2, 2:-2]
            wet = (want[..., 0] > 1e-2) & (h > 1e-2)
            if wet.any():
                worst = max(worst, float(np.abs((h + b) - (want[..., 0] + b))[wet].max()))
    print(f"fp32 deviation, bench hierarchy: max surface difference {worst:.3e} m", flush=True)
    assert worst <= 1e-5


def test_device_plans_equal_the_host_plans(gpu):
    # swe_amr_plans (built on the device from the rectangle tables) against
    # amr.fill_plan and amr.average_plan (the host plans the CPU tests pin to
    # the reference coupling), byte for byte, before and after a regrid
    L, AmrSolver, torch = gpu
    from paper_1901_06798_amd import amr
    cases = [W.amr_three_levels(2, bed="shelf", amp=2.0), W.amr_three_levels(4, bed="shelf"),
             W.amr_nested()]
    for H in cases:
        print(f"case device plans ratio={H.ratio} patches={len(H.patches)}", flush=True)
        s = AmrSolver(H, L.params())
        for regridded in (False, True):
            if regridded:
                s.set_dt(6.0)
                s.run(2)
                s.regrid(tol=0.05 if H.ratio != 4 else 0.5)
            for lev in range(1, s.nlev):
                f = amr.fill_plan(s.geo[lev], s.geo[lev - 1], s.r)
                a = amr.average_plan(s.geo[lev], s.geo[lev - 1], s.r)
                assert np.array_equal(s.fill_ops[lev].cpu().numpy(), f.view(np.uint8)), lev
                assert np.array_equal(s.avg_ops[lev - 1].cpu().numpy(), a.view(np.uint8)), lev
