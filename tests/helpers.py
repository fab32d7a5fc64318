"""Small test helpers: embedding workload problems into the reference solver's
layout and running it to a given time."""
from __future__ import annotations

import numpy as np


def oracle_setup(O, pb):
    q, b = O.new_state(pb.h, pb.hu, pb.hv, pb.b)
    g = O.grid(pb.mx, pb.my, pb.dx, pb.dy, pb.bc)
    O.ghost_fill_b(g, b)
    O.ghost_fill(g, q)
    return g, q, b


def oracle_run_to(O, P, g, q, b, T):
    """Advance with the CFL rule and shorten the last step to land on T."""
    t = 0.0
    dt = 0.0
    n = 0
    while True:
        O.ghost_fill(g, q)
        sm = O.speed_scan(P, g, q, b)
        rate = max(sm[0] / g.dx, sm[1] / g.dy)
        dt = P.cfl_desired / rate
        if t + dt >= T:
            dt = T - t
            O.run(P, g, q, b, 1, dt_forced=[dt])
            return T, n + 1
        O.run(P, g, q, b, 1, dt_forced=[dt])
        t += dt
        n += 1


def interior(q):
    return q[2:-2, 2:-2]
