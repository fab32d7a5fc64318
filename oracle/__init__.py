"""Reference FP64 CPU solver for the shallow water patch step.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package; the library under
``paper_1901_06798_amd`` never does.  The C source (``swe_oracle.c``) follows
Sec. 2 of Qin, LeVeque & Motley (the shallow water equations, the
wave-propagation form with limited second-order corrections, dimensional
splitting and the CFL condition), plus a written-out reading of the augmented
Riemann solver that the paper cites but does not state.

State layout: numpy arrays ``q`` of shape ``(my + 4, mx + 4, 3)`` holding
``(h, hu, hv)`` per cell (array of structures, two ghost layers), and ``b`` of
shape ``(my + 4, mx + 4)``.

Parity status of each function is listed in the test suite's oracle pins
(tests/test_oracle_*.py); the unsplit (transverse) mode is pinned only by
invariants (lake at rest, mass, symmetry, convergence), not by a closed form.
"""
from __future__ import annotations

import contextlib
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "swe_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

BC_WALL, BC_EXTRAP, BC_USER = 0, 1, 2
EDGE_WET, EDGE_WALL_R, EDGE_WALL_L, EDGE_DRY = 0, 1, 2, 3


_OPC_SRC = os.path.join(_HERE, "opcount.cpp")
_OPC_PATH = os.path.join(_HERE, "liboracle_opcount.so")


def build(verbose: bool = False) -> str:
    """Compile the oracle with gcc (plain -O3, no fast-math, no FP contraction),
    and its operation-counting build (opcount.cpp: the same source as C++
    with a counting real type, single-threaded)."""
    cmd = ["gcc", "-std=c11", "-O3", "-fPIC", "-shared", "-fopenmp",
           "-ffp-contract=off", "-fno-fast-math", "-Wall", "-Wextra",
           "-Wno-unused-parameter", _SRC, "-o", _LIB_PATH + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(_LIB_PATH + ".tmp", _LIB_PATH)
    # -fpermissive: the C source converts malloc's void * implicitly
    cmd = ["g++", "-std=c++17", "-O2", "-fPIC", "-shared", "-fpermissive", "-w",
           "-ffp-contract=off", "-fno-fast-math", _OPC_SRC, "-o", _OPC_PATH + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(_OPC_PATH + ".tmp", _OPC_PATH)
    return _LIB_PATH


class Params(ctypes.Structure):
    _fields_ = [("g", ctypes.c_double), ("drytol", ctypes.c_double),
                ("manning_n", ctypes.c_double), ("cfl_desired", ctypes.c_double),
                ("cfl_max", ctypes.c_double), ("h_corr", ctypes.c_double),
                ("method", ctypes.c_int32),
                ("order", ctypes.c_int32), ("transverse_order", ctypes.c_int32),
                ("pad_", ctypes.c_int32)]


class Grid(ctypes.Structure):
    _fields_ = [("mx", ctypes.c_int32), ("my", ctypes.c_int32),
                ("dx", ctypes.c_double), ("dy", ctypes.c_double),
                ("bc", ctypes.c_int32 * 4)]


class Waves(ctypes.Structure):
    _fields_ = [("z", (ctypes.c_double * 3) * 3), ("s", ctypes.c_double * 3),
                ("kind", ctypes.c_int32), ("clamped", ctypes.c_int32),
                ("shallow", ctypes.c_int32), ("pad_", ctypes.c_int32)]


_lib = None
_D = ctypes.POINTER(ctypes.c_double)


def _bind(L):
    P, G = ctypes.POINTER(Params), ctypes.POINTER(Grid)
    d, i32, i64 = ctypes.c_double, ctypes.c_int32, ctypes.c_int64
    L.orc_riemann.argtypes = [P] + [d] * 8 + [ctypes.POINTER(Waves)]
    L.orc_riemann.restype = None
    L.orc_fluctuations.argtypes = [ctypes.POINTER(Waves), _D, _D]
    L.orc_mc_limiter.argtypes = [d]
    L.orc_mc_limiter.restype = d
    L.orc_ghost_fill.argtypes = [G, _D]
    L.orc_ghost_fill_b.argtypes = [G, _D]
    L.orc_step.argtypes = [P, G, _D, _D, d, _D, _D, ctypes.POINTER(i32)]
    L.orc_step.restype = i64
    L.orc_step_sphere.argtypes = [P, G, _D, _D, d, _D, _D, _D, _D, ctypes.POINTER(i32)]
    L.orc_step_sphere.restype = i64
    L.orc_speed_scan.argtypes = [P, G, _D, _D, _D]
    L.orc_run.argtypes = [P, G, _D, _D, i32, d, _D, _D, ctypes.POINTER(i32),
                          ctypes.POINTER(i32)]
    L.orc_run.restype = i64
    L.orc_mass.argtypes = [G, _D]
    L.orc_mass.restype = d
    L.orc_set_threads.argtypes = [i32]
    L.orc_get_threads.restype = i32
    return L


_opc = None


def opcount_lib():
    """The operation-counting build (same functions, single-threaded, plus
    orc_opcount_get / orc_opcount_reset)."""
    global _opc
    if _opc is None:
        if not os.path.exists(_OPC_PATH):
            build()
        L = _bind(ctypes.CDLL(_OPC_PATH))
        L.orc_opcount_get.argtypes = [ctypes.POINTER(ctypes.c_int64)]
        L.orc_opcount_get.restype = None
        L.orc_opcount_reset.restype = None
        _opc = L
    return _opc


OPCOUNT_KINDS = ("add", "mul", "div", "sqrt", "cmp", "other")


def opcount_reset() -> None:
    opcount_lib().orc_opcount_reset()


def opcount_get() -> dict:
    """Operations counted by the counting build since the last reset:
    add (additions and subtractions), mul, div, sqrt, cmp (comparisons of
    reals), other (sign flips, absolute values, powers); "flops" is the
    first four summed."""
    buf = (ctypes.c_int64 * 6)()
    opcount_lib().orc_opcount_get(buf)
    out = dict(zip(OPCOUNT_KINDS, (int(v) for v in buf)))
    out["flops"] = out["add"] + out["mul"] + out["div"] + out["sqrt"]
    return out


@contextlib.contextmanager
def counting():
    """Inside the block, every call of this module runs on the counting build
    (single-threaded; results bit for bit the plain build's); the counters
    start at zero.  Read them with opcount_get()."""
    global _lib
    saved = _lib
    _lib = opcount_lib()
    opcount_reset()
    try:
        yield
    finally:
        _lib = saved


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        _lib = _bind(ctypes.CDLL(_LIB_PATH))
    return _lib


def params(g=9.81, drytol=1e-3, manning_n=0.0, cfl_desired=0.9, cfl_max=1.0,
           h_corr=0.1, method=0, order=2, transverse_order=2) -> Params:
    return Params(g, drytol, manning_n, cfl_desired, cfl_max, h_corr, method, order,
                  transverse_order, 0)


def grid(mx, my, dx, dy, bc=(BC_WALL,) * 4) -> Grid:
    return Grid(mx, my, dx, dy, (ctypes.c_int32 * 4)(*bc))


def _ptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_D)


def set_threads(n: int) -> None:
    lib().orc_set_threads(int(n))


def get_threads() -> int:
    return int(lib().orc_get_threads())


def mc_limiter(theta: float) -> float:
    return float(lib().orc_mc_limiter(float(theta)))


def riemann(left, right, p: Params | None = None):
    """Solve one edge.  left/right = (h, normal momentum, transverse momentum, b).

    Returns (Z, s, kind, clamped) with Z[p, k] the f-wave p in components
    (mass, normal momentum, transverse momentum)."""
    p = p or params()
    w = Waves()
    lib().orc_riemann(ctypes.byref(p), *[float(v) for v in left],
                      *[float(v) for v in right], ctypes.byref(w))
    Z = np.array([[w.z[a][k] for k in range(3)] for a in range(3)])
    s = np.array([w.s[a] for a in range(3)])
    return Z, s, int(w.kind), int(w.clamped)


def fluctuations(left, right, p: Params | None = None):
    p = p or params()
    w = Waves()
    lib().orc_riemann(ctypes.byref(p), *[float(v) for v in left],
                      *[float(v) for v in right], ctypes.byref(w))
    am = np.zeros(3)
    ap = np.zeros(3)
    lib().orc_fluctuations(ctypes.byref(w), _ptr(am), _ptr(ap))
    return am, ap


def new_state(h, hu, hv, b, bc=(BC_WALL,) * 4):
    """Embed interior (my, mx) arrays into ghost-framed AoS arrays; fill ghosts."""
    my, mx = np.shape(h)
    q = np.zeros((my + 4, mx + 4, 3))
    q[2:-2, 2:-2, 0] = h
    q[2:-2, 2:-2, 1] = hu
    q[2:-2, 2:-2, 2] = hv
    bb = np.zeros((my + 4, mx + 4))
    bb[2:-2, 2:-2] = b
    return q, bb


def ghost_fill(g: Grid, q: np.ndarray) -> None:
    lib().orc_ghost_fill(ctypes.byref(g), _ptr(q))


def ghost_fill_b(g: Grid, b: np.ndarray) -> None:
    lib().orc_ghost_fill_b(ctypes.byref(g), _ptr(b))


def step(p: Params, g: Grid, q: np.ndarray, b: np.ndarray, dt: float):
    """One step from q (ghosts must be filled).  Returns (q_out, smax, clamps, nonfinite)."""
    out = np.empty_like(q)
    smax = np.zeros(2)
    nf = ctypes.c_int32(0)
    c = lib().orc_step(ctypes.byref(p), ctypes.byref(g), _ptr(q), _ptr(b), float(dt),
                       _ptr(out), _ptr(smax), ctypes.byref(nf))
    return out, smax, int(c), int(nf.value)


def sphere_metric(lat0_deg: float, dlat_deg: float, my: int, bc=None):
    """Capacities kap[j] (rows j = 0 .. my + 3 of the ghost frame) and edge
    length ratios len[e] = cos(latitude of the edge between rows e - 1 and e),
    e = 0 .. my + 4, of a latitude-longitude patch whose first interior row
    starts at latitude lat0_deg (rows are dlat_deg high).  The capacity is the
    cell area over its area at the equator: (sin phi_top - sin phi_bottom) /
    dphi.  With bc (xlo, xhi, ylo, yhi), a wall at ylo or yhi makes the two
    ghost rows beyond it the mirror image of the interior rows inside it, in
    geometry as in state (the reflection that defines a wall ghost cell): their
    kap and len are the mirrored interior values.  Then the x-sweep moves a
    ghost row exactly as its image row, the Riemann problem at the wall stays
    symmetric, and no mass crosses the wall; with the geometric values beyond
    the wall it would."""
    d = np.deg2rad(dlat_deg)
    edge = np.array([np.deg2rad(lat0_deg + (j - 2) * dlat_deg) for j in range(my + 5)])
    kap = np.array([(np.sin(edge[j + 1]) - np.sin(edge[j])) / d for j in range(my + 4)])
    ln = np.array([np.cos(edge[e]) for e in range(my + 5)])
    if bc is not None and bc[2] == BC_WALL:
        # rows 1, 0 reflect rows 2, 3 about edge 2
        kap[1], kap[0] = kap[2], kap[3]
        ln[1], ln[0] = ln[3], ln[4]
    if bc is not None and bc[3] == BC_WALL:
        # rows my + 2, my + 3 reflect rows my + 1, my about edge my + 2
        kap[my + 2], kap[my + 3] = kap[my + 1], kap[my]
        ln[my + 3], ln[my + 4] = ln[my + 1], ln[my]
    return kap, ln


def step_sphere(p: Params, g: Grid, q: np.ndarray, b: np.ndarray, dt: float, kap, ln):
    """One split step of a latitude-longitude patch (g.dx, g.dy: R dlon, R dlat).
    Returns (q_out, smax, clamps, nonfinite)."""
    out = np.empty_like(q)
    smax = np.zeros(2)
    nf = ctypes.c_int32(0)
    k = np.ascontiguousarray(kap, dtype=np.float64)
    ln_ = np.ascontiguousarray(ln, dtype=np.float64)
    c = lib().orc_step_sphere(ctypes.byref(p), ctypes.byref(g), _ptr(q), _ptr(b), float(dt),
                              _ptr(k), _ptr(ln_), _ptr(out), _ptr(smax), ctypes.byref(nf))
    return out, smax, int(c), int(nf.value)


def speed_scan(p: Params, g: Grid, q: np.ndarray, b: np.ndarray):
    smax = np.zeros(2)
    lib().orc_speed_scan(ctypes.byref(p), ctypes.byref(g), _ptr(q), _ptr(b), _ptr(smax))
    return smax


def run(p: Params, g: Grid, q: np.ndarray, b: np.ndarray, nsteps: int, dt0: float = 0.0,
        dt_forced=None):
    """Advance q in place.  Returns dict(dt, clamps, retakes, nonfinite)."""
    dts = np.zeros(max(nsteps, 1))
    rt = ctypes.c_int32(0)
    nf = ctypes.c_int32(0)
    forced = None
    if dt_forced is not None:
        forced = np.ascontiguousarray(dt_forced, dtype=np.float64)
        assert forced.size >= nsteps
    c = lib().orc_run(ctypes.byref(p), ctypes.byref(g), _ptr(q), _ptr(b), int(nsteps),
                      float(dt0), _ptr(forced) if forced is not None else None,
                      _ptr(dts), ctypes.byref(rt), ctypes.byref(nf))
    return {"dt": dts[:nsteps], "clamps": int(c), "retakes": int(rt.value),
            "nonfinite": int(nf.value)}


def mass(g: Grid, q: np.ndarray) -> float:
    return float(lib().orc_mass(ctypes.byref(g), _ptr(q)))
