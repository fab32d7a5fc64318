"""The library's flag clustering (swe_amr_cluster, host code) against the
reference clustering: the same boxes in the same order, on seeded fields of
blobs and noise, on degenerate fields, and across the efficiency and
minimum-side settings (integer work: exact equality)."""
import numpy as np
import pytest

from oracle import regrid as G
from paper_1901_06798_amd import _lib as L


def field(seed, my=40, mx=56, k=4, noise=0.02):
    rng = np.random.default_rng(seed)
    F = np.zeros((my, mx), dtype=bool)
    Y, X = np.mgrid[0:my, 0:mx]
    for _ in range(k):
        cx, cy = rng.integers(0, mx), rng.integers(0, my)
        rx, ry = rng.integers(1, 10, 2)
        F |= ((X - cx) / rx) ** 2 + ((Y - cy) / ry) ** 2 <= 1.0
    F |= rng.random((my, mx)) < noise
    return F


@pytest.mark.parametrize("seed", range(12))
@pytest.mark.parametrize("eff,min_side", [(0.7, 2), (0.9, 1), (0.5, 3), (1.0, 2)])
def test_library_clustering_equals_the_reference(seed, eff, min_side):
    F = field(seed)
    assert L.swe_amr_cluster(F.astype(np.uint8), eff, min_side) == G.cluster(F, eff, min_side)


@pytest.mark.parametrize("shape", [(1, 1), (1, 30), (30, 1), (7, 9)])
def test_degenerate_fields(shape):
    F = np.zeros(shape, dtype=bool)
    assert L.swe_amr_cluster(F.astype(np.uint8)) == [] == G.cluster(F)
    F[...] = True
    assert L.swe_amr_cluster(F.astype(np.uint8)) == G.cluster(F) == [
        (0, 0, shape[1] - 1, shape[0] - 1)]
    F[...] = False
    F.flat[::3] = True
    assert L.swe_amr_cluster(F.astype(np.uint8), 0.8, 1) == G.cluster(F, 0.8, 1)


def test_many_boxes_and_bad_arguments():
    rng = np.random.default_rng(1)
    F = rng.random((64, 64)) < 0.05     # sparse noise: many small boxes (> 64)
    got = L.swe_amr_cluster(F.astype(np.uint8), 0.9, 1)
    assert got == G.cluster(F, 0.9, 1) and len(got) > 64
    lib = L.lib()
    import ctypes
    n = ctypes.c_int32(0)
    f = np.zeros((4, 4), dtype=np.uint8)
    assert lib.swe_amr_cluster(f.ctypes.data, 4, 4, 3, 0.7, 2, None, 0, ctypes.byref(n)) == \
        L.SWE_EINVAL  # pitch < mx
    assert lib.swe_amr_cluster(f.ctypes.data, 4, 4, 4, 0.0, 2, None, 0, ctypes.byref(n)) == \
        L.SWE_EINVAL  # efficiency
