"""GPU parity of the unsplit step with transverse waves (FP64) against the
reference solver's unsplit mode, 1e-12 relative per field."""
import numpy as np
import pytest

from paper_1901_06798_amd import workloads as W
from test_gpu_split import compare, run_pair, smooth_random_problem

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


def test_unsplit_hump(gpu, orc):
    pb = W.gaussian_hump(100, 2000.0)
    s, st, dts, qref, r = run_pair(gpu, orc, pb, 40, method=1)
    compare(st, qref)
    np.testing.assert_allclose(dts, r["dt"], rtol=1e-13)
    h = st[0]
    assert np.abs(h - h.T).max() < 1e-9  # symmetric under x <-> y


@pytest.mark.parametrize("tr", [1, 2])
@pytest.mark.parametrize("mx,my,bc", [
    (61, 67, (W.BC_EXTRAP,) * 4),
    (130, 45, (W.BC_WALL, W.BC_EXTRAP, W.BC_WALL, W.BC_EXTRAP)),
    (9, 70, (W.BC_WALL,) * 4),
])
def test_unsplit_ragged_wet_dry(gpu, orc, mx, my, bc, tr):
    pb = smooth_random_problem(mx, my, seed=300 + mx + my, bc=bc)
    s, st, dts, qref, r = run_pair(gpu, orc, pb, 20, method=1, transverse_order=tr)
    compare(st, qref)


def test_unsplit_lake_at_rest(gpu):
    L, PatchSolver, torch = gpu
    pb = W.shelf_grid(120, 500.0, seed=11, amp=0.0, x_s_frac=0.5, width=5e3)
    s = PatchSolver(pb, L.params(method=1))
    s.run(20)
    h, hu, hv = s.state()
    assert np.array_equal(h, pb.h) and not hu.any() and not hv.any()
