"""The precision study at full size (2048^2 walled shelf, dx 500 m, the
2 m source 60 km seaward of the shelf break, 2000 steps): the FP32
surface-deviation step and, as the floor that FP32 storage alone sets, the
same step with FP64 arithmetic over FP32 storage (SWE_F32_STORE), both driven
by the FP64 run's step sizes; and the FP64 run started from the FP32-rounded
initial state (one rounding, no more).  Errors: max |surface difference|
against the FP64 run over cells wet (h > 1e-2 m) in both.

Bars: FP32 within 1e-5 m while the wave crosses open water (steps 250, 500,
750); after the run-up onto the dry coast (the surface reaches ~10 m) the
workload amplifies rounding-size differences by orders of magnitude, and FP32
stays within 10x of the FP32-storage floor at every checkpoint.  The stricter
reading, within 3x of the one-rounding floor, is recorded as an expected
failure with the measured ratio."""
import numpy as np
import pytest

from paper_1901_06798_amd import workloads as W

pytestmark = pytest.mark.gpu
EVERY = 250


@pytest.fixture(scope="module")
def study():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1901_06798_amd import _lib as L
    from paper_1901_06798_amd.solver import PatchSolver
    n, steps = 2048, 2000
    pb = W.shelf_walls(n=n, dx=1024e3 / n, seed=4, nsteps=steps)
    sea = L.params().sea_level
    b32 = pb.b.astype(np.float32).astype(np.float64)
    eta32 = np.where(pb.h > 0.0, pb.h + pb.b - sea, pb.b - sea).astype(np.float32)
    pbc = W.Problem(pb.name + "_rounded", np.where(pb.h > 0.0, np.maximum(
        eta32.astype(np.float64) + sea - b32, 0.0), 0.0), pb.hu, pb.hv, b32, pb.dx, pb.dy, pb.bc)
    print(f"case precision study {n}^2 walled shelf, {steps} steps", flush=True)
    s64 = PatchSolver(pb, L.params())
    s32 = PatchSolver(pb, L.params(precision=L.F32_DEV))
    sst = PatchSolver(pb, L.params(precision=L.F32_STORE))
    s64c = PatchSolver(pbc, L.params())
    s64.initial_dt()
    dt_log = torch.zeros(steps, dtype=torch.float64, device=s64.dev)

    def err(a, b_):
        ha, hb = a.state()[0], b_.state()[0]
        both = (ha > 1e-2) & (hb > 1e-2)
        return float(np.abs(a.surface() - b_.surface())[both].max())

    rows, surf = [], 0.0
    for k0 in range(0, steps, EVERY):
        for k in range(k0, k0 + EVERY):
            dt_log[k].copy_(s64.dt[0])
            s64.enqueue_step(retake=False)
            for s in (s32, sst, s64c):
                s.enqueue_step(dt_log.data_ptr() + 8 * k, cfl=False)
                s.smax.zero_()
        torch.cuda.synchronize()
        rows.append((k0 + EVERY, err(s32, s64), err(sst, s64), err(s64c, s64)))
        print("step %d: fp32 %.3e, fp32 storage %.3e, one rounding %.3e" % rows[-1], flush=True)
        surf = max(surf, float(np.abs(s64.surface()[s64.state()[0] > 1e-2]).max()))
    flags = (s64.flags(), s32.flags())
    return rows, surf, flags


def test_open_water_within_1e5_m(study):
    rows, surf, flags = study
    assert flags[0] == (0, 0)
    for step, e32, _, _ in rows:
        if step <= 750:
            assert e32 <= 1e-5, (step, e32)


def test_after_run_up_within_10x_of_the_fp32_storage_floor(study):
    rows, surf, flags = study
    assert surf > 5.0  # the wave did run up the coast (largest surface over the checkpoints)
    for step, e32, est, _ in rows:
        assert e32 <= 10.0 * max(est, 1e-5), (step, e32, est)


@pytest.mark.xfail(reason="after the run-up FP32 storage re-rounds the state every step; the "
                          "one-rounding floor does not: measured FP32 / one-rounding floor "
                          "= 53 at step 1000, 15 at step 2000 (FP32 storage with FP64 "
                          "arithmetic: 10 and 20)", strict=False)
def test_after_run_up_within_3x_of_the_one_rounding_floor(study):
    rows, surf, flags = study
    for step, e32, _, e1 in rows:
        if step > 750:
            assert e32 <= 3.0 * e1, (step, e32, e1)
