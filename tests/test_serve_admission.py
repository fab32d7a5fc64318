"""Admission order of the serving loop (host logic, no GPU): oldest first,
later requests pass one that does not fit for a bounded time."""
from types import SimpleNamespace

from paper_1901_06798_amd.serve import admit_in_order


def reqs(*sizes_and_arrivals):
    return [SimpleNamespace(rid=k, size=s, arrival=t) for k, (s, t) in enumerate(sizes_and_arrivals)]


def budget(free):
    state = {"free": free}

    def try_admit(sc):
        if sc.size <= state["free"]:
            state["free"] -= sc.size
            return True
        return False
    return try_admit, state


def test_strict_arrival_order_without_bypass():
    q = reqs((8, 0.0), (1, 0.1), (1, 0.2))
    try_admit, st = budget(4)
    assert admit_in_order(q, try_admit, now=0.3, max_bypass_s=0.0) == []
    assert [sc.rid for sc in q] == [0, 1, 2] and st["free"] == 4


def test_later_requests_pass_one_that_does_not_fit():
    q = reqs((8, 0.0), (1, 0.1), (5, 0.2), (2, 0.25))
    try_admit, st = budget(4)
    got = admit_in_order(q, try_admit, now=0.3, max_bypass_s=0.5)
    # 1 and 2 fit (3 of 4 units), 5 does not; the head stays first in line
    assert [sc.rid for sc in got] == [1, 3]
    assert [sc.rid for sc in q] == [0, 2] and st["free"] == 1


def test_a_request_waiting_past_the_bound_holds_the_line():
    q = reqs((8, 0.0), (1, 0.1), (1, 0.2))
    try_admit, st = budget(4)
    assert admit_in_order(q, try_admit, now=0.6, max_bypass_s=0.5) == []
    # a blocked request inside the bound is passed, one past it stops the scan
    q = reqs((1, 0.0), (8, 0.05), (1, 0.4), (8, 0.45), (1, 0.5))
    try_admit, st = budget(4)
    got = admit_in_order(q, try_admit, now=0.6, max_bypass_s=0.5)
    assert [sc.rid for sc in got] == [0]
    assert [sc.rid for sc in q] == [1, 2, 3, 4]


def test_everything_that_fits_is_admitted_in_arrival_order():
    q = reqs((1, 0.0), (2, 0.1), (1, 0.2))
    try_admit, st = budget(10)
    got = admit_in_order(q, try_admit, now=0.3, max_bypass_s=0.5)
    assert [sc.rid for sc in got] == [0, 1, 2] and q == [] and st["free"] == 6
