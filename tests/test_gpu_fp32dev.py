"""GPU tests of the FP32 surface-deviation path: FP32 storage of
eta' = h + b - sea_level, FP64 solves at shallow and dry edges (SWE_F32_DEV),
or FP64 arithmetic throughout over the same storage (SWE_F32_STORE).  Bars: a
lake at rest stays exactly at rest; the surface stays within 1e-5 m of the
FP64 reference (driven by the FP64 step sizes) on cells wet in both runs."""
import numpy as np
import pytest

from helpers import interior, oracle_setup
from paper_1901_06798_amd import workloads as W

pytestmark = pytest.mark.gpu
ETA_TOL = 1e-5  # metres


@pytest.fixture(scope="module")
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1901_06798_amd import _lib as L
    from paper_1901_06798_amd.solver import PatchSolver
    L.lib()
    return L, PatchSolver, torch


@pytest.mark.parametrize("prec", ["F32_DEV", "F32_STORE"])
def test_lake_at_rest_is_exact_in_fp32(gpu, prec):
    L, PatchSolver, torch = gpu
    pb = W.shelf_grid(200, 500.0, seed=13, amp=0.0, x_s_frac=0.5, width=5e3)
    assert (pb.h == 0).any()
    s = PatchSolver(pb, L.params(precision=getattr(L, prec)))
    s.run(40)
    torch.cuda.synchronize()
    Q = s.planes().cpu().numpy()[:, 2:-2, 2: pb.mx + 2]
    wet = pb.h > 0
    assert np.all(Q[0][wet] == 0.0)  # eta' of wet cells stays exactly 0
    assert not Q[1].any() and not Q[2].any()
    assert s.flags() == (0, 0)


def surface_error(h32, eta32, h64, eta64, wet_min=1e-2):
    both = (h32 > wet_min) & (h64 > wet_min)
    return np.abs(eta32 - eta64)[both].max(), int(((h32 > 1e-3) != (h64 > 1e-3)).sum())


@pytest.mark.parametrize("prec", ["F32_DEV", "F32_STORE"])
def test_surface_error_against_reference(gpu, orc, prec):
    """Shelf with a coast, walls, 400 steps: FP32 storage vs the FP64
    reference solver with the same step sizes."""
    L, PatchSolver, torch = gpu
    pb = W.shelf_walls(n=192, dx=2000.0, seed=4, nsteps=400)
    s64 = PatchSolver(pb, L.params())
    dts = s64.run(400)
    g, q, b = oracle_setup(orc, pb)
    orc.run(orc.params(), g, q, b, 400, dt_forced=dts)
    s32 = PatchSolver(pb, L.params(precision=getattr(L, prec)))
    s32.run_forced(dts)
    torch.cuda.synchronize()
    h32, _, _ = s32.state()
    eta32 = s32.surface()
    h64 = interior(q)[..., 0]
    eta64 = h64 + interior(b)
    err, mismatch = surface_error(h32, eta32, h64, eta64)
    print(f"{prec} surface error {err:.3e} m, wet/dry mismatches {mismatch}", flush=True)
    assert err <= ETA_TOL
    # the FP64 GPU run itself is the reference solver's result
    for a, k in zip(s64.state(), range(3)):
        ref = interior(q)[..., k]
        assert np.abs(a - ref).max() <= 1e-12 * np.abs(ref).max()


def test_fp32_mass_drift_small(gpu):
    L, PatchSolver, torch = gpu
    pb = W.shelf_walls(n=256, dx=2000.0, seed=4, nsteps=300)
    s = PatchSolver(pb, L.params(precision=L.F32_DEV))
    m0 = s.mass()
    s.run(300)
    torch.cuda.synchronize()
    m1 = s.mass()
    assert abs(m1 - m0) / m0 < 1e-7
    assert s.flags()[0] & (L.STATUS_NONFINITE | L.STATUS_NEG_DEPTH) == 0
