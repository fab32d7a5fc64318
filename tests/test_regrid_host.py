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


def test_init_plan_matches_cell_by_cell_rule():
    # the rectangle-by-rectangle plan against the rule applied to every cell:
    # the first old patch of the level whose interior holds the cell gives a
    # copy, else the first patch below whose interior holds (I // r, J // r)
    import numpy as np
    from paper_1901_06798_amd import _lib as L
    from paper_1901_06798_amd import amr as A

    class G(A._Geo):
        def __init__(self, rects, pad):
            self.i0 = np.array([q[0] for q in rects], dtype=np.int64)
            self.j0 = np.array([q[1] for q in rects], dtype=np.int64)
            self.mx = np.array([q[2] for q in rects], dtype=np.int64)
            self.my = np.array([q[3] for q in rects], dtype=np.int64)
            self.pitch = self.mx + pad
            sizes = (self.my + 4) * self.pitch
            self.off = np.concatenate([[0], np.cumsum(sizes)[:-1]]).astype(np.int64)

    rng = np.random.default_rng(5)
    for _ in range(60):
        r = int(rng.choice([2, 4]))
        crs = [(0, 0, 30, 30)] if rng.random() < 0.5 else [(0, 0, 18, 30), (15, 0, 15, 30),
                                                             (5, 5, 10, 10)]
        coarse = G(crs, 8)

        def rects(n):
            out = []
            for _ in range(n):
                mx, my = int(rng.integers(1, 25)), int(rng.integers(1, 25))
                out.append((int(rng.integers(0, 30 * r - mx)), int(rng.integers(0, 30 * r - my)),
                            mx, my))
            return out
        new = G(rects(int(rng.integers(1, 4))), 4)
        orr = rects(int(rng.integers(0, 5)))
        old = G(orr, 6) if orr else None
        ops = A.init_plan(new, old, coarse, r)
        n = 0
        for k in range(len(new.i0)):
            for jj in range(new.my[k]):
                for ii in range(new.mx[k]):
                    I, J = new.i0[k] + ii, new.j0[k] + jj
                    e = ops[n]
                    n += 1
                    assert e["dst"] == new.off[k] + (jj + 2) * new.pitch[k] + ii + 2
                    src = next((s for s in range(len(old.i0)) if old.i0[s] <= I < old.i0[s] + old.mx[s]
                                and old.j0[s] <= J < old.j0[s] + old.my[s]), None) if old else None
                    if src is not None:
                        assert e["kind"] == L.SWE_AMR_COPY
                        assert e["src"] == old.elem(src, I, J)
                        continue
                    Ic, Jc = I // r, J // r
                    c = next(s for s in range(len(coarse.i0))
                             if coarse.i0[s] <= Ic < coarse.i0[s] + coarse.mx[s]
                             and coarse.j0[s] <= Jc < coarse.j0[s] + coarse.my[s])
                    assert e["kind"] == L.SWE_AMR_COARSE and e["src"] == coarse.elem(c, Ic, Jc)
        assert n == ops.size
