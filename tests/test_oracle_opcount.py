"""The oracle's operation counter (oracle/opcount.cpp: the reference solver
compiled with a counting real type): it leaves every result bit for bit as
the plain build computes it, counts a known function exactly (the MC limiter:
1 addition, 2 multiplications, 3 comparisons), counts no arithmetic for a
Riemann problem with two dry sides, and on a uniform sea its count per step
grows by the same amount for each equal widening of the patch (the work of a
uniform column of cells is the same wherever the column is added)."""
import numpy as np

import oracle as O
from paper_1901_06798_amd import workloads as W


def run_plain_and_counted(pb, nsteps):
    P = O.params()
    out = []
    for counted in (False, True):
        q, b = O.new_state(pb.h, pb.hu, pb.hv, pb.b)
        g = O.grid(pb.mx, pb.my, pb.dx, pb.dy, pb.bc)
        O.ghost_fill_b(g, b)
        if counted:
            with O.counting():
                r = O.run(P, g, q, b, nsteps)
                ops = O.opcount_get()
        else:
            r = O.run(P, g, q, b, nsteps)
            ops = None
        out.append((q, r, ops))
    return out


def test_counting_build_leaves_results_bitwise():
    for pb in (W.gaussian_hump(n=40, dx=2000.0, sigma=15e3),
               W.shelf_grid(48, 2000.0, seed=1, amp=3.0, name="shelf48")):
        (q0, r0, _), (q1, r1, ops) = run_plain_and_counted(pb, 12)
        assert np.array_equal(q0, q1)
        assert np.array_equal(r0["dt"], r1["dt"])
        assert r0["clamps"] == r1["clamps"]
        assert ops["flops"] > 0 and ops["div"] > 0 and ops["sqrt"] > 0


def test_limiter_and_dry_edge_counts():
    with O.counting():
        O.mc_limiter(0.25)
        c = O.opcount_get()
    assert (c["add"], c["mul"], c["div"], c["sqrt"], c["cmp"], c["other"]) == (1, 2, 0, 0, 3, 0)
    with O.counting():
        O.riemann((0.0, 0.0, 0.0, 5.0), (0.0, 0.0, 0.0, 7.0))
        c = O.opcount_get()
    assert c["flops"] == 0 and c["other"] == 0


def test_uniform_sea_count_is_affine_in_width():
    P = O.params()
    counts = []
    for mx in (10, 20, 30):
        h = np.full((12, mx), 50.0)
        z = np.zeros_like(h)
        q, b = O.new_state(h, z, z, np.full_like(h, -50.0))
        g = O.grid(mx, 12, 100.0, 100.0)
        O.ghost_fill_b(g, b)
        O.ghost_fill(g, q)
        with O.counting():
            O.step(P, g, q, b, 0.5)
            counts.append(O.opcount_get())
    for k in ("add", "mul", "div", "sqrt", "cmp"):
        assert counts[2][k] - counts[1][k] == counts[1][k] - counts[0][k] > 0, k
