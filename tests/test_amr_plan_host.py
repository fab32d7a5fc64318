"""Host checks of the AMR ghost-cell plan (no GPU): amr.fill_plan, evaluated
by the rule that swe.h states for swe_amr_fill (a plain loop over the entries
on pool-shaped host arrays), gives cell for cell what the reference coupling
gives (oracle/amr.py fill).  This pins the plan's stencil offsets, weights and
copy/coarse choices; the device kernel then only has to follow the stated
rule, which the GPU tests check."""
import numpy as np
import pytest

import oracle as O
from oracle import amr as A
from oracle import regrid as G
from paper_1901_06798_amd import _lib as L
from paper_1901_06798_amd import amr
from paper_1901_06798_amd import workloads as W


class Pool:
    """A level's patches packed as a BatchedSolver lays them out (pitch padded
    to 16 elements, patch sizes to 64), three state planes and a bed plane."""

    def __init__(self, patches):
        self.offs, self.layout, t = [], [], 0
        for p in patches:
            pitch = -(-(p.mx + 4) // 16) * 16
            size = -(-(pitch * (p.my + 4)) // 64) * 64
            self.offs.append(t)
            self.layout.append((pitch, size))
            t += size
        self.plane = t
        self.geo = amr._Geo(patches, self)
        self.patches = patches

    def pack(self, arrays, nplanes):
        """Flat planes from per-patch (my + 4, mx + 4[, nplanes]) arrays."""
        out = np.zeros(nplanes * self.plane)
        for k, (p, a) in enumerate(zip(self.patches, arrays)):
            pitch = self.layout[k][0]
            a = a.reshape(p.my + 4, p.mx + 4, nplanes)
            for c in range(nplanes):
                v = out[c * self.plane + self.offs[k]: c * self.plane + self.offs[k]
                        + pitch * (p.my + 4)].reshape(p.my + 4, pitch)
                v[:, : p.mx + 4] = a[..., c]
        return out

    def unpack(self, flat, k):
        p, pitch = self.patches[k], self.layout[k][0]
        out = np.zeros((p.my + 4, p.mx + 4, 3))
        for c in range(3):
            v = flat[c * self.plane + self.offs[k]: c * self.plane + self.offs[k]
                     + pitch * (p.my + 4)].reshape(p.my + 4, pitch)
            out[..., c] = v[:, : p.mx + 4]
        return out


def apply_fill(ops, qf, psf, bf, qcopy, pscopy, qco, qcn, psc, bc, alpha, drytol):
    """The rule of swe_amr_fill as swe.h states it, entry by entry."""
    w0, w1 = 1.0 - alpha, alpha
    for op in ops:
        dst = int(op["dst"])
        if op["kind"] == L.SWE_AMR_COPY:
            for c in range(3):
                qf[dst + c * psf] = qcopy[int(op["src"]) + c * pscopy]
            continue

        def at(k):
            return (w0 * (qco[k] + bc[k]) + w1 * (qcn[k] + bc[k]),
                    w0 * qco[k + psc] + w1 * qcn[k + psc],
                    w0 * qco[k + 2 * psc] + w1 * qcn[k + 2 * psc])
        wx, wy = float(op["wx"]), float(op["wy"])
        used = [0] + ([1] if wx > 0 else []) + ([2] if wy > 0 else []) + (
            [3] if wx > 0 and wy > 0 else [])
        st = [int(v) for v in op["st"]]
        if all(st[k] >= 0 and qco[st[k]] > drytol and qcn[st[k]] > drytol for k in used):
            c = {k: at(st[k]) for k in used}
            v = []
            for m in range(3):
                line0 = (1.0 - wx) * c[0][m]
                if wx > 0:
                    line0 = line0 + wx * c[1][m]
                val = (1.0 - wy) * line0
                if wy > 0:
                    line1 = (1.0 - wx) * c[2][m]
                    if wx > 0:
                        line1 = line1 + wx * c[3][m]
                    val = val + wy * line1
                v.append(val)
        else:
            s = int(op["src"])
            if qco[s] <= drytol and qcn[s] <= drytol:
                for c in range(3):
                    qf[dst + c * psf] = 0.0
                continue
            v = at(s)
        d = v[0] - bf[dst]
        h = d if d > 0.0 else 0.0
        qf[dst] = h
        qf[dst + psf] = 0.0 if h <= drytol else v[1]
        qf[dst + 2 * psf] = 0.0 if h <= drytol else v[2]


@pytest.fixture(scope="module")
def P():
    O.lib()
    return O.params()


@pytest.mark.parametrize("ratio", [1, 2, 4])
@pytest.mark.parametrize("alpha_k", [0, 1])
def test_ghost_plan_by_the_stated_rule_equals_the_reference_fill(P, ratio, alpha_k):
    H = W.amr_three_levels(ratio, bed="shelf", amp=2.0, u0=0.3, n1=32)
    h = A.Hierarchy(H, P)
    h.run(6.0, 1)
    for lev in (2, 3):
        coarse = h.levels[lev - 2]
        old = [p.q.copy() for p in coarse]
        for p in coarse:  # a new coarse state: one more step of the level below
            if lev == 2:
                O.ghost_fill(p.g, p.q)
            out, _, _, _ = O.step(P, p.g, p.q, p.b, 6.0 / ratio ** (lev - 2))
            p.q[2:-2, 2:-2] = out[2:-2, 2:-2]
        alpha = alpha_k / max(ratio, 2)
        fine = h.levels[lev - 1]
        pc, pf = Pool(coarse), Pool(fine)
        ops = amr.fill_plan(pf.geo, pc.geo, ratio)
        qf = pf.pack([p.q for p in fine], 3)
        bf = pf.pack([p.b for p in fine], 1)
        qco = pc.pack(old, 3)
        qcn = pc.pack([p.q for p in coarse], 3)
        bc = pc.pack([p.b for p in coarse], 1)
        apply_fill(ops, qf, pf.plane, bf, qf.copy(), pf.plane, qco, qcn, pc.plane, bc, alpha,
                   P.drytol)
        h.fill(lev, old, alpha)
        nlin = 0
        for k, p in enumerate(fine):
            got = pf.unpack(qf, k)
            assert np.array_equal(got, p.q), (ratio, lev, k)
        coarse_ops = ops[ops["kind"] == L.SWE_AMR_COARSE]
        nlin = int(np.sum(np.all(coarse_ops["st"] >= 0, axis=1)))
        assert coarse_ops.size > 0 and nlin > 0
