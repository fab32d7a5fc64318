"""Absolute-performance metrics of a run from its timeline (Qin, LeVeque &
Motley, Sec. 5, the metrics P1, P2, P3).

With Omega_X the union of the time intervals of all events of kind X (GPU
computation, CPU computation, host-to-device and device-to-host copies) and
E_total the interval the program runs:

    P1 = |Omega_GPU| / |E_total|
    P2 = |Omega_CPU| / |E_total|
    P3 = |(Omega_h2d U Omega_d2h) - (Omega_CPU U Omega_GPU)| / |E_total|

P3 is the share of the run spent in copies that overlap no computation (the
printed formula is garbled; this is its reading: the set difference of the
copy intervals and the computation intervals, over the run's length).

The intervals come from a rocprofv3 trace of the run (kernel dispatches,
memory copies and ROCTx ranges): `Markers` names the host's computation
phases and the run's extent as ROCTx ranges ("host: ..." and the outer range
given to `from_rocprof`), which the trace records on the same clock as the
device events.  Without the ROCTx library the markers do nothing.

    python -m paper_1901_06798_amd.timeline <trace dir> [outer range name]
"""
from __future__ import annotations

import contextlib
import csv
import ctypes
import glob
import json
import os
import sys

HOST_PREFIX = "host:"


# ---------------------------------------------------------------------------
# interval arithmetic (closed intervals [a, b], a <= b, in any time unit)

def merge(intervals):
    """Disjoint, sorted intervals covering the same set as `intervals`."""
    out = []
    for a, b in sorted((float(a), float(b)) for a, b in intervals if b > a):
        if out and a <= out[-1][1]:
            if b > out[-1][1]:
                out[-1][1] = b
        else:
            out.append([a, b])
    return [(a, b) for a, b in out]


def measure(intervals) -> float:
    """|U intervals|: the total length of their union."""
    return sum(b - a for a, b in merge(intervals))


def clip(intervals, lo: float, hi: float):
    """The parts of `intervals` inside [lo, hi]."""
    return [(max(a, lo), min(b, hi)) for a, b in intervals if min(b, hi) > max(a, lo)]


def difference(a_intervals, b_intervals):
    """(U a) - (U b) as disjoint intervals."""
    a = merge(a_intervals)
    b = merge(b_intervals)
    out = []
    j = 0
    for lo, hi in a:
        cur = lo
        while j < len(b) and b[j][1] <= cur:
            j += 1
        k = j
        while k < len(b) and b[k][0] < hi:
            if b[k][0] > cur:
                out.append((cur, b[k][0]))
            cur = max(cur, b[k][1])
            if cur >= hi:
                break
            k += 1
        if cur < hi:
            out.append((cur, hi))
    return out


def p_metrics(gpu, cpu, h2d, d2h, total) -> dict:
    """P1, P2, P3 of a run whose extent is the interval `total`; every event
    list is first clipped to it."""
    lo, hi = total
    span = hi - lo
    if not span > 0:
        raise ValueError("the run's extent has no length")
    g, c = clip(gpu, lo, hi), clip(cpu, lo, hi)
    copies = clip(list(h2d) + list(d2h), lo, hi)
    return {"P1": measure(g) / span, "P2": measure(c) / span,
            "P3": measure(difference(copies, g + c)) / span, "span": span}


# ---------------------------------------------------------------------------
# ROCTx ranges

class Markers:
    """ROCTx ranges through the rocprofiler-sdk ROCTx library, if it loads."""

    def __init__(self):
        self.lib = None
        for name in ("librocprofiler-sdk-roctx.so.1", "librocprofiler-sdk-roctx.so",
                     "/opt/rocm/lib/librocprofiler-sdk-roctx.so"):
            try:
                lib = ctypes.CDLL(name)
            except OSError:
                continue
            lib.roctxRangePushA.argtypes = [ctypes.c_char_p]
            lib.roctxRangePushA.restype = ctypes.c_int
            lib.roctxRangePop.restype = ctypes.c_int
            self.lib = lib
            break

    @contextlib.contextmanager
    def range(self, name: str):
        if self.lib is None:
            yield
            return
        self.lib.roctxRangePushA(name.encode())
        try:
            yield
        finally:
            self.lib.roctxRangePop()


_markers = None


def markers() -> Markers:
    global _markers
    if _markers is None:
        _markers = Markers()
    return _markers


# ---------------------------------------------------------------------------
# rocprofv3 CSV traces

def _rows(trace_dir: str, suffix: str):
    rows = []
    for path in sorted(glob.glob(os.path.join(trace_dir, "**", f"*{suffix}"), recursive=True)):
        with open(path, newline="") as f:
            rows.extend(csv.DictReader(f))
    return rows


def _span(r) -> tuple:
    return (float(r["Start_Timestamp"]), float(r["End_Timestamp"]))


def _marker_name(r) -> str:
    for key in ("Function", "Message", "Name", "Marker_Name"):
        if r.get(key):
            return r[key]
    return ""


def from_rocprof(trace_dir: str, outer: str = "serve") -> dict:
    """P1-P3 from the kernel, memory-copy and marker traces of a rocprofv3
    CSV run (`--kernel-trace --memory-copy-trace --marker-trace
    --output-format csv`).  The run's extent is the union of the ROCTx ranges
    named `outer` (from the first start to the last end); CPU computation is
    the ranges named "host: ..."."""
    kernels = [_span(r) for r in _rows(trace_dir, "kernel_trace.csv")]
    copies = _rows(trace_dir, "memory_copy_trace.csv")
    h2d, d2h = [], []
    for r in copies:
        d = " ".join(str(v) for k, v in r.items() if "irection" in k or k == "Kind")
        if "HOST_TO_DEVICE" in d:
            h2d.append(_span(r))
        elif "DEVICE_TO_HOST" in d:
            d2h.append(_span(r))
    marks = [(_marker_name(r), _span(r)) for r in _rows(trace_dir, "marker_api_trace.csv")]
    outer_spans = [s for n, s in marks if n == outer]
    if not outer_spans:
        raise ValueError(f"no ROCTx range named {outer!r} in {trace_dir}")
    total = (min(a for a, _ in outer_spans), max(b for _, b in outer_spans))
    cpu = [s for n, s in marks if n.startswith(HOST_PREFIX)]
    out = p_metrics(kernels, cpu, h2d, d2h, total)
    out.update({"span_ms": out.pop("span") * 1e-6, "kernels": len(kernels), "h2d": len(h2d),
                "d2h": len(d2h), "host_ranges": len(cpu), "outer_ranges": len(outer_spans)})
    return out


if __name__ == "__main__":
    if len(sys.argv) < 2:
        print(__doc__)
        sys.exit(2)
    print(json.dumps(from_rocprof(sys.argv[1], *(sys.argv[2:3] or ["serve"]))))
