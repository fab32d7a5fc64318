"""GPU tests of regridding (swe_amr_flag on the device, swe_amr_cluster on
the host, swe_amr_init, AmrSolver.regrid) against the reference regridding:
the device flags equal the reference flags of the same state bit for bit; a
regrid from the initial state gives the reference's rectangles and the
reference's new cells exactly, and the regridded hierarchy then runs as the
reference does (FP64, relative 1e-12)."""
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


def reference(H):
    import oracle as O
    from oracle import amr as A
    O.lib()
    return A.Hierarchy(H, O.params()), O


def test_device_flags_equal_the_reference_flags(gpu):
    L, AmrSolver, torch = gpu
    from oracle import regrid as G
    H = W.amr_three_levels(2, bed="shelf", amp=2.0, u0=0.3)
    s = AmrSolver(H, L.params())
    s.set_dt(6.0)
    s.run(2)
    print("case device flags after 2 coarse steps", flush=True)
    for lev in (1, 2):
        bs = s.levels[lev - 1]
        fh = s.refine_flags(lev).cpu().numpy()
        nflag = 0
        for k, p in enumerate(s.lpatches[lev - 1]):
            pitch, off = bs.layout[k][0], bs.offs[k]
            got = fh[off: off + pitch * (p.my + 4)].reshape(p.my + 4, pitch)[2:-2, 2: p.mx + 2]
            h, hu, hv = s.state(lev, k)
            q = np.zeros((p.my + 4, p.mx + 4, 3))
            q[2:-2, 2:-2, 0], q[2:-2, 2:-2, 1], q[2:-2, 2:-2, 2] = h, hu, hv
            want = G.flag_patch(q, p.b_frame, 5e-3, 1e-3, 2, 1)
            assert np.array_equal(got.astype(bool), want), (lev, k)
            nflag += int(want.sum())
        assert nflag > 0


@pytest.mark.parametrize("ratio", [2, 4])
def test_regrid_matches_the_reference(gpu, ratio):
    L, AmrSolver, torch = gpu
    from oracle import regrid as G
    H = W.amr_three_levels(ratio, bed="shelf", amp=2.0, u0=0.3)
    print(f"case regrid from the initial state ratio={ratio}", flush=True)
    s = AmrSolver(H, L.params())
    got = s.regrid()
    h, O = reference(H)
    want = G.regrid(h, H)
    assert got == want
    assert len(got[1]) > 0 and len(got) == 3
    for lev in (2, 3):
        for k, p in enumerate(h.levels[lev - 1]):
            st = s.state(lev, k)
            for c in range(3):
                assert np.array_equal(st[c], p.q[2:-2, 2:-2, c]), (lev, k, c)
    # and the regridded hierarchy runs as the reference
    s.set_dt(6.0)
    s.run(2)
    torch.cuda.synchronize()
    h.run(6.0, 2)
    assert s.flags() == (0, 0)
    for lev in range(1, 4):
        pats = h.levels[lev - 1]
        scale = [max(np.abs(p.q[2:-2, 2:-2, c]).max() for p in pats) for c in range(3)]
        for k, p in enumerate(pats):
            st = s.state(lev, k)
            for c in range(3):
                err = np.abs(st[c] - p.q[2:-2, 2:-2, c]).max() / max(scale[c], 1e-300)
                assert err <= 1e-12, (lev, k, c, err)


def test_regrid_of_a_sea_at_rest_removes_the_finer_levels(gpu):
    L, AmrSolver, torch = gpu
    H = W.amr_three_levels(2, bed="bowl", amp=0.0)
    s = AmrSolver(H, L.params())
    assert s.regrid() == [[(0, 0, H.n1, H.n1)]]
    assert s.nlev == 1
    s.set_dt(6.0)
    s.run(2)
    torch.cuda.synchronize()
    h, hu, hv = s.state(1, 0)
    assert not hu.any() and not hv.any()
