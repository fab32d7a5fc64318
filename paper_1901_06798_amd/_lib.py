"""ctypes binding of the C ABI in include/swe.h (argument marshalling only).

Every function has the C name and argument order; device pointers are passed
as Python ints (e.g. ``tensor.data_ptr()``) and the stream as an int
(``torch.cuda.current_stream().cuda_stream``) or 0.  A non-zero return code
raises SweError with the library's message.  If the HIP library has not been
built, importing the binding fails loudly: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes

import numpy as np
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("SWE_LIB_PATH", os.path.join(_HERE, "libswe.so"))

SWE_OK, SWE_EINVAL, SWE_EHIP = 0, -1, -2
STATUS_NEG_DEPTH, STATUS_NONFINITE, STATUS_CFL_EXCEEDED, STATUS_RETAKEN = 1, 2, 4, 8
SPLIT, UNSPLIT = 0, 1
F64, F32_DEV, F32_STORE = 0, 1, 2
BC_WALL, BC_EXTRAP, BC_USER = 0, 1, 2
SWE_AMR_COPY, SWE_AMR_COARSE = 0, 1


class SweError(RuntimeError):
    pass


class swe_params(ctypes.Structure):
    _fields_ = [("g", ctypes.c_double), ("drytol", ctypes.c_double),
                ("h_corr", ctypes.c_double), ("manning_n", ctypes.c_double),
                ("cfl_desired", ctypes.c_double), ("cfl_max", ctypes.c_double),
                ("sea_level", ctypes.c_double), ("h_fp64", ctypes.c_double),
                ("method", ctypes.c_int32), ("order", ctypes.c_int32),
                ("transverse_order", ctypes.c_int32), ("precision", ctypes.c_int32)]


class swe_patch(ctypes.Structure):
    _fields_ = [("off", ctypes.c_int64), ("plane_stride", ctypes.c_int64),
                ("dx", ctypes.c_double), ("dy", ctypes.c_double),
                ("mx", ctypes.c_int32), ("my", ctypes.c_int32), ("pitch", ctypes.c_int32),
                ("group", ctypes.c_int32), ("tref", ctypes.c_int32), ("level", ctypes.c_int32),
                ("bc", ctypes.c_int8 * 4), ("reserved", ctypes.c_int32)]


assert ctypes.sizeof(swe_patch) == 64


class swe_schedule(ctypes.Structure):
    _fields_ = [("seg", ctypes.c_int32), ("rows_per_task", ctypes.c_int32),
                ("waves_per_group", ctypes.c_int32), ("per_substep", ctypes.c_int32),
                ("order", ctypes.c_int32), ("groups_per_cu", ctypes.c_int32)]


class swe_launch(ctypes.Structure):
    _fields_ = [("rows_per_task", ctypes.c_int32), ("waves_per_block", ctypes.c_int32),
                ("xcd_run", ctypes.c_int32), ("reserved", ctypes.c_int32)]


def launch(rows_per_task=0, waves_per_block=0, xcd_run=0) -> swe_launch:
    return swe_launch(rows_per_task, waves_per_block, xcd_run, 0)


class swe_task(ctypes.Structure):
    _fields_ = [("patch", ctypes.c_int32), ("strip", ctypes.c_int32), ("row0", ctypes.c_int32),
                ("rows", ctypes.c_int32), ("col0", ctypes.c_int32), ("lanes", ctypes.c_int32)]


class swe_item(ctypes.Structure):
    _fields_ = [("task_begin", ctypes.c_int32), ("task_end", ctypes.c_int32),
                ("patch", ctypes.c_int32), ("substeps", ctypes.c_int32)]


def schedule(seg=64, rows_per_task=0, waves_per_group=4, per_substep=0, order=0,
             groups_per_cu=0) -> swe_schedule:
    return swe_schedule(seg, rows_per_task, waves_per_group, per_substep, order, groups_per_cu)


def params(g=9.81, drytol=1e-3, h_corr=0.1, manning_n=0.0, cfl_desired=0.9, cfl_max=1.0,
           sea_level=0.0, h_fp64=1.0, method=SPLIT, order=2, transverse_order=2,
           precision=F64) -> swe_params:
    return swe_params(g, drytol, h_corr, manning_n, cfl_desired, cfl_max, sea_level, h_fp64,
                      method, order, transverse_order, precision)


def patch(mx, my, pitch, dx, dy, off=0, plane_stride=None, group=0, tref=1, level=1,
          bc=(BC_WALL,) * 4) -> swe_patch:
    if plane_stride is None:
        plane_stride = pitch * (my + 4)
    return swe_patch(off, plane_stride, dx, dy, mx, my, pitch, group, tref, level,
                     (ctypes.c_int8 * 4)(*bc), 0)


_lib = None
_P = ctypes.c_void_p


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise SweError(f"HIP library {LIB_PATH} is not built; run __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        i32 = ctypes.c_int32
        pp = ctypes.POINTER(swe_params)
        L.swe_patch_step.argtypes = [pp, ctypes.POINTER(swe_patch), _P, _P, _P, _P, _P, _P, _P]
        L.swe_ghost_fill.argtypes = [pp, _P, i32, i32, i32, _P, _P, i32, _P]
        L.swe_speed_scan.argtypes = [pp, _P, i32, i32, i32, _P, _P, _P, _P]
        L.swe_cfl_reduce.argtypes = [pp, _P, i32, i32, _P, _P, _P, _P, _P, i32, _P]
        L.swe_patch_retake.argtypes = [pp, ctypes.POINTER(swe_patch), _P, _P, _P, _P, _P, _P,
                                       _P, _P]
        L.swe_mass.argtypes = [pp, _P, i32, _P, _P, _P, _P]
        L.swe_level_steps.argtypes = [_P, i32, i32, _P, _P]
        i64, dbl = ctypes.c_int64, ctypes.c_double
        pl = ctypes.POINTER(swe_launch)
        L.swe_patch_tasks.argtypes = [ctypes.POINTER(swe_patch), pl]
        L.swe_patch_tasks.restype = i32
        L.swe_workspace_bytes.argtypes = [ctypes.POINTER(swe_patch), pl]
        L.swe_workspace_bytes.restype = ctypes.c_size_t
        L.swe_patch_step_sched.argtypes = [pp, ctypes.POINTER(swe_patch), _P, _P, _P, _P, _P, _P,
                                           _P, i64, pl, _P]
        L.swe_patch_order.argtypes = [ctypes.POINTER(swe_patch), _P, i64, pl, _P]
        L.swe_patch_step_sphere.argtypes = [pp, ctypes.POINTER(swe_patch), _P, _P, _P, _P, _P,
                                            _P, _P, _P, i64, pl, _P]
        L.swe_patch_retake_sphere.argtypes = [pp, ctypes.POINTER(swe_patch), _P, _P, _P, _P, _P,
                                              _P, _P, _P, _P]
        L.swe_patch_step_cfl.argtypes = [pp, ctypes.POINTER(swe_patch), _P, _P, _P, _P, _P, _P,
                                         _P, _P, _P, _P, i64, ctypes.POINTER(swe_launch), _P]
        L.swe_patch_retake_cfl.argtypes = [pp, ctypes.POINTER(swe_patch), _P, _P, _P, _P, _P, _P,
                                           _P, _P, _P, i32, _P]
        L.swe_amr_plans.argtypes = [_P, i32, _P, i32, i32, i64, _P, _P, _P, _P, _P, _P]
        L.swe_speed_scan_sphere.argtypes = [pp, _P, i32, i32, _P, _P, _P, _P, _P]
        L.swe_mass_sphere.argtypes = [pp, _P, _P, _P, _P, _P]
        L.swe_state_import.argtypes = [pp, _P, i32, i32, i32, _P, _P, i64, i64, _P, _P, _P]
        L.swe_state_export.argtypes = [pp, _P, i32, i32, i32, _P, _P, _P, i64, i64, _P]
        L.swe_amr_fill.argtypes = [pp, _P, i64, _P, i64, _P, _P, _P, i64, _P, dbl, _P]
        L.swe_amr_average.argtypes = [pp, _P, i64, i32, _P, i64, _P, _P, i64, _P, _P]
        L.swe_amr_flag.argtypes = [pp, _P, i32, i32, i32, _P, _P, dbl, i32, i32, _P, _P]
        L.swe_amr_cluster.argtypes = [_P, i32, i32, i32, dbl, i32, _P, i32,
                                      ctypes.POINTER(i32)]
        L.swe_amr_init.argtypes = [pp, i32, _P, i32, i64, _P, i64, _P, _P, i32, _P, i64, _P, i32,
                                   _P, i64, _P, _P]
        ps = ctypes.POINTER(swe_schedule)
        pi32 = ctypes.POINTER(i32)
        L.swe_batched_plan.argtypes = [_P, i32, ps, _P, pi32, _P, pi32, pi32, pi32]
        L.swe_batched_step.argtypes = [pp, _P, _P, i32, _P, _P, i32, i32, _P, _P, _P, i64, _P,
                                       _P, _P, _P, _P, _P, ps, _P]
        L.swe_batched_retake.argtypes = [pp, _P, _P, i32, _P, _P, i32, i32, _P, _P, _P, i64,
                                         _P, _P, _P, _P, _P, _P, ps, _P, i32, _P]
        L.swe_batched_advance.argtypes = [pp, _P, i32, i32, _P, i32, _P, _P, i32, i32, _P, _P,
                                          i32, _P, i64, _P, _P, _P, _P, _P, _P, _P, _P, _P,
                                          ps, i32, _P]
        L.swe_batched_step_static.argtypes = [pp, _P, _P, i32, _P, _P, i32, i32, _P, _P, i64,
                                              _P, _P, _P, _P, _P, ps, _P]
        L.swe_last_error.restype = ctypes.c_char_p
        L.swe_version.restype = ctypes.c_char_p
        for name in ("swe_patch_step", "swe_ghost_fill", "swe_speed_scan", "swe_cfl_reduce",
                     "swe_mass", "swe_batched_plan", "swe_batched_step", "swe_patch_retake",
                     "swe_batched_retake", "swe_patch_step_sched", "swe_patch_order",
                     "swe_amr_fill", "swe_amr_average", "swe_amr_flag", "swe_amr_cluster",
                     "swe_amr_init", "swe_patch_step_sphere", "swe_state_import",
                     "swe_state_export", "swe_batched_step_static", "swe_level_steps",
                     "swe_patch_retake_sphere", "swe_speed_scan_sphere", "swe_mass_sphere",
                     "swe_batched_advance", "swe_patch_step_cfl", "swe_patch_retake_cfl",
                     "swe_amr_plans"):
            getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def _check(rc: int, what: str) -> None:
    if rc != SWE_OK:
        msg = lib().swe_last_error().decode()
        raise SweError(f"{what} failed ({rc}): {msg}")


def swe_version() -> str:
    return lib().swe_version().decode()


def swe_patch_step(p: swe_params, pt: swe_patch, q_in: int, q_out: int, b: int, dt: int,
                   smax: int, status: int, stream: int = 0) -> None:
    _check(lib().swe_patch_step(ctypes.byref(p), ctypes.byref(pt), q_in, q_out, b, dt, smax,
                                status, stream), "swe_patch_step")


def _lp(launch: swe_launch | None):
    return ctypes.byref(launch) if launch is not None else None


def swe_patch_tasks(pt: swe_patch, launch: swe_launch | None = None) -> int:
    n = lib().swe_patch_tasks(ctypes.byref(pt), _lp(launch))
    if n < 0:
        _check(n, "swe_patch_tasks")
    return n


def swe_workspace_bytes(pt: swe_patch, launch: swe_launch | None = None) -> int:
    return int(lib().swe_workspace_bytes(ctypes.byref(pt), _lp(launch)))


def swe_patch_step_sched(p: swe_params, pt: swe_patch, q_in: int, q_out: int, b: int, dt: int,
                         smax: int, status: int, sched: int, sched_len: int,
                         launch: swe_launch | None = None, stream: int = 0) -> None:
    _check(lib().swe_patch_step_sched(ctypes.byref(p), ctypes.byref(pt), q_in, q_out, b, dt,
                                      smax, status, sched, sched_len, _lp(launch), stream),
           "swe_patch_step_sched")


def swe_patch_step_sphere(p: swe_params, pt: swe_patch, q_in: int, q_out: int, b: int, dt: int,
                          smax: int, status: int, metric: int, sched: int = 0,
                          sched_len: int = 0, launch: swe_launch | None = None,
                          stream: int = 0) -> None:
    _check(lib().swe_patch_step_sphere(ctypes.byref(p), ctypes.byref(pt), q_in, q_out, b, dt,
                                       smax, status, metric, sched, sched_len, _lp(launch),
                                       stream), "swe_patch_step_sphere")


def swe_patch_order(pt: swe_patch, sched: int, sched_len: int,
                    launch: swe_launch | None = None, stream: int = 0) -> None:
    _check(lib().swe_patch_order(ctypes.byref(pt), sched, sched_len, _lp(launch), stream),
           "swe_patch_order")


def swe_level_steps(dt_coarse: int, ratio: int, nlevels: int, dt_levels: int,
                    stream: int = 0) -> None:
    _check(lib().swe_level_steps(dt_coarse, ratio, nlevels, dt_levels, stream),
           "swe_level_steps")


def swe_state_import(p: swe_params, patches: int, n: int, max_mx: int, max_my: int, src: int,
                     src_b: int, q: int, b: int, stream: int = 0, src_shift: int = 0,
                     src_stride: int = 0) -> None:
    _check(lib().swe_state_import(ctypes.byref(p), patches, n, max_mx, max_my, src, src_b,
                                  src_shift, src_stride, q, b, stream), "swe_state_import")


def swe_state_export(p: swe_params, patches: int, n: int, max_mx: int, max_my: int, q: int,
                     b: int, dst: int, stream: int = 0, dst_shift: int = 0,
                     dst_stride: int = 0) -> None:
    _check(lib().swe_state_export(ctypes.byref(p), patches, n, max_mx, max_my, q, b, dst,
                                  dst_shift, dst_stride, stream), "swe_state_export")


def swe_amr_fill(p: swe_params, ops: int, nops: int, q_fine: int, fine_plane_stride: int,
                 b_fine: int, q_coarse_old: int, q_coarse_new: int, coarse_plane_stride: int,
                 b_coarse: int, alpha: float, stream: int = 0) -> None:
    _check(lib().swe_amr_fill(ctypes.byref(p), ops, nops, q_fine, fine_plane_stride, b_fine,
                              q_coarse_old, q_coarse_new, coarse_plane_stride, b_coarse,
                              float(alpha), stream), "swe_amr_fill")


def swe_amr_average(p: swe_params, ops: int, nops: int, ratio: int, q_fine: int,
                    fine_plane_stride: int, b_fine: int, q_coarse: int,
                    coarse_plane_stride: int, b_coarse: int, stream: int = 0) -> None:
    _check(lib().swe_amr_average(ctypes.byref(p), ops, nops, ratio, q_fine, fine_plane_stride,
                                 b_fine, q_coarse, coarse_plane_stride, b_coarse, stream),
           "swe_amr_average")


def swe_amr_flag(p: swe_params, patches: int, n: int, max_mx: int, max_my: int, q: int, b: int,
                 tol: float, buffer: int, margin: int, flags: int, stream: int = 0) -> None:
    _check(lib().swe_amr_flag(ctypes.byref(p), patches, n, max_mx, max_my, q, b, float(tol),
                              buffer, margin, flags, stream), "swe_amr_flag")


def swe_amr_cluster(flags, efficiency: float = 0.7, min_side: int = 2):
    """Boxes (i0, j0, i1, j1) of a host uint8 array flags[j, i] (C order)."""
    f = np.ascontiguousarray(flags, dtype=np.uint8)
    my, mx = f.shape
    n = ctypes.c_int32(0)
    cap = 64
    while True:
        out = np.zeros(4 * cap, dtype=np.int32)
        rc = lib().swe_amr_cluster(f.ctypes.data, mx, my, mx, float(efficiency), min_side,
                                   out.ctypes.data, cap, ctypes.byref(n))
        if rc == SWE_OK:
            return [tuple(int(v) for v in out[4 * k: 4 * k + 4]) for k in range(n.value)]
        if n.value <= cap:
            _check(rc, "swe_amr_cluster")
        cap = n.value


# swe_amr_rect as a numpy record (the C layout: off, i0, j0, mx, my, pitch,
# reserved)
AMR_RECT_DTYPE = np.dtype([("off", "<i8"), ("i0", "<i4"), ("j0", "<i4"), ("mx", "<i4"),
                           ("my", "<i4"), ("pitch", "<i4"), ("reserved", "<i4")])


def swe_amr_init(p: swe_params, ratio: int, new_rects: int, n_new: int, max_cells: int,
                 q_new: int, new_plane_stride: int, b_new: int, old_rects: int, n_old: int,
                 q_old: int, old_plane_stride: int, coarse_rects: int, n_coarse: int,
                 q_coarse: int, coarse_plane_stride: int, b_coarse: int, stream: int = 0) -> None:
    _check(lib().swe_amr_init(ctypes.byref(p), ratio, new_rects, n_new, max_cells, q_new,
                              new_plane_stride, b_new, old_rects, n_old, q_old,
                              old_plane_stride, coarse_rects, n_coarse, q_coarse,
                              coarse_plane_stride, b_coarse, stream),
           "swe_amr_init")


def swe_amr_plans(fine: int, n_fine: int, coarse: int, n_coarse: int, ratio: int,
                  max_entries: int, fill_ops: int, fill_first: int, avg_ops: int, avg_first: int,
                  err: int, stream: int = 0) -> None:
    _check(lib().swe_amr_plans(fine, n_fine, coarse, n_coarse, ratio, max_entries, fill_ops,
                               fill_first, avg_ops, avg_first, err, stream), "swe_amr_plans")


def swe_ghost_fill(p: swe_params, patches: int, n: int, max_mx: int, max_my: int, q: int,
                   b: int, fill_b: int, stream: int = 0) -> None:
    _check(lib().swe_ghost_fill(ctypes.byref(p), patches, n, max_mx, max_my, q, b, fill_b,
                                stream), "swe_ghost_fill")


def swe_speed_scan(p: swe_params, patches: int, n: int, max_mx: int, max_my: int, q: int,
                   b: int, smax_patch: int, stream: int = 0) -> None:
    _check(lib().swe_speed_scan(ctypes.byref(p), patches, n, max_mx, max_my, q, b, smax_patch,
                                stream), "swe_speed_scan")


def swe_cfl_reduce(p: swe_params, patches: int, n: int, ngroups: int, smax_patch: int,
                   dt_group: int, status: int, group_flags: int, initial: int,
                   stream: int = 0, retake: int = 0) -> None:
    _check(lib().swe_cfl_reduce(ctypes.byref(p), patches, n, ngroups, smax_patch, dt_group,
                                status, group_flags, retake, initial, stream), "swe_cfl_reduce")


def swe_patch_retake(p: swe_params, pt: swe_patch, q_in: int, q_out: int, b: int, dt: int,
                     smax: int, status: int, retake: int, stream: int = 0) -> None:
    _check(lib().swe_patch_retake(ctypes.byref(p), ctypes.byref(pt), q_in, q_out, b, dt, smax,
                                  status, retake, stream), "swe_patch_retake")


def swe_patch_step_cfl(p: swe_params, pt: swe_patch, q_in: int, q_out: int, b: int, dt: int,
                       smax: int, status: int, retake: int, counter: int, metric: int = 0,
                       sched: int = 0, sched_len: int = 0, launch: swe_launch | None = None,
                       stream: int = 0) -> None:
    _check(lib().swe_patch_step_cfl(ctypes.byref(p), ctypes.byref(pt), q_in, q_out, b, dt, smax,
                                    status, retake, counter, metric, sched, sched_len,
                                    ctypes.byref(launch) if launch is not None else None, stream),
           "swe_patch_step_cfl")


def swe_patch_retake_cfl(p: swe_params, pt: swe_patch, q_in: int, q_out: int, b: int, dt: int,
                         smax: int, status: int, retake: int, counter: int, metric: int = 0,
                         last: int = 1, stream: int = 0) -> None:
    _check(lib().swe_patch_retake_cfl(ctypes.byref(p), ctypes.byref(pt), q_in, q_out, b, dt,
                                      smax, status, retake, counter, metric, last, stream),
           "swe_patch_retake_cfl")


def swe_patch_retake_sphere(p: swe_params, pt: swe_patch, q_in: int, q_out: int, b: int,
                            dt: int, smax: int, status: int, metric: int, retake: int,
                            stream: int = 0) -> None:
    _check(lib().swe_patch_retake_sphere(ctypes.byref(p), ctypes.byref(pt), q_in, q_out, b, dt,
                                         smax, status, metric, retake, stream),
           "swe_patch_retake_sphere")


def swe_speed_scan_sphere(p: swe_params, patch: int, max_mx: int, max_my: int, q: int, b: int,
                          metric: int, smax: int, stream: int = 0) -> None:
    _check(lib().swe_speed_scan_sphere(ctypes.byref(p), patch, max_mx, max_my, q, b, metric,
                                       smax, stream), "swe_speed_scan_sphere")


def swe_mass_sphere(p: swe_params, patch: int, q: int, metric: int, mass: int,
                    stream: int = 0) -> None:
    _check(lib().swe_mass_sphere(ctypes.byref(p), patch, q, metric, mass, stream),
           "swe_mass_sphere")


def swe_mass(p: swe_params, patches: int, n: int, q: int, b: int, mass_patch: int,
             stream: int = 0) -> None:
    _check(lib().swe_mass(ctypes.byref(p), patches, n, q, b, mass_patch, stream), "swe_mass")


def swe_batched_plan(patches, sched: swe_schedule):
    """Plan for a host list of swe_patch; returns a Plan: ctypes arrays items and
    tasks with the counts nitems, ntasks, nplain (the last nplain tasks are
    the plain ones) and nsub (launches of the plain tasks)."""
    n = len(patches)
    arr = (swe_patch * n)(*patches)
    ni = ctypes.c_int32(0)
    nt = ctypes.c_int32(0)
    npl = ctypes.c_int32(0)
    nsb = ctypes.c_int32(0)
    _check(lib().swe_batched_plan(ctypes.addressof(arr), n, ctypes.byref(sched), None,
                                  ctypes.byref(ni), None, ctypes.byref(nt), ctypes.byref(npl),
                                  ctypes.byref(nsb)), "swe_batched_plan")
    items = (swe_item * max(ni.value, 1))()
    tasks = (swe_task * max(nt.value, 1))()
    _check(lib().swe_batched_plan(ctypes.addressof(arr), n, ctypes.byref(sched),
                                  ctypes.addressof(items), ctypes.byref(ni),
                                  ctypes.addressof(tasks), ctypes.byref(nt), ctypes.byref(npl),
                                  ctypes.byref(nsb)), "swe_batched_plan")
    return Plan(items, ni.value, tasks, nt.value, npl.value, nsb.value)


class Plan:
    def __init__(self, items, nitems, tasks, ntasks, nplain, nsub):
        self.items, self.nitems, self.tasks, self.ntasks = items, nitems, tasks, ntasks
        self.nplain, self.nsub = nplain, nsub

    def device(self, dev):
        """(items, tasks) as uint8 device tensors."""
        import torch
        to = lambda a: torch.frombuffer(bytearray(bytes(a)), dtype=torch.uint8).to(dev)
        return to(self.items), to(self.tasks)


SWE_TASK_BYTES = ctypes.sizeof(swe_task)


def swe_batched_advance(p: swe_params, patches: int, npatches: int, ngroups: int, items: int,
                        nitems: int, tasks: int, plain: int, nplain: int, nsub: int, pool_0: int,
                        pool_1: int, first: int, pool_work: int, pool_elems: int, pool_b: int,
                        dt_group: int, smax_patch: int, status: int, group_status: int,
                        group_flags: int, retake: int, pending: int, queue: int,
                        sched: swe_schedule, nsteps: int, stream: int = 0) -> None:
    _check(lib().swe_batched_advance(ctypes.byref(p), patches, npatches, ngroups, items, nitems,
                                     tasks, plain, nplain, nsub, pool_0, pool_1, first,
                                     pool_work, pool_elems, pool_b, dt_group, smax_patch,
                                     status, group_status, group_flags, retake, pending, queue,
                                     ctypes.byref(sched), nsteps, stream),
           "swe_batched_advance")


def swe_batched_step(p: swe_params, patches: int, items: int, nitems: int, tasks: int,
                     plain: int, nplain: int, nsub: int, pool_in: int, pool_out: int,
                     pool_work: int, pool_elems: int, pool_b: int, dt_group: int,
                     smax_patch: int, status: int, queue: int, sched: swe_schedule,
                     stream: int = 0, group_status: int = 0) -> None:
    _check(lib().swe_batched_step(ctypes.byref(p), patches, items, nitems, tasks, plain, nplain,
                                  nsub, pool_in, pool_out, pool_work, pool_elems, pool_b,
                                  dt_group, smax_patch, status, group_status, queue,
                                  ctypes.byref(sched), stream), "swe_batched_step")


SWE_STATIC_WORK_BYTES = 32 * 1024 * 1024


def swe_batched_step_static(p: swe_params, patches: int, items: int, nitems: int, tasks: int,
                            plain: int, nplain: int, nsub: int, pool_in: int, pool_out: int,
                            pool_elems: int, pool_b: int, dt_group: int, smax_patch: int,
                            status: int, sched: swe_schedule, stream: int = 0,
                            group_status: int = 0) -> None:
    _check(lib().swe_batched_step_static(ctypes.byref(p), patches, items, nitems, tasks, plain,
                                         nplain, nsub, pool_in, pool_out, pool_elems, pool_b,
                                         dt_group, smax_patch, status, group_status,
                                         ctypes.byref(sched), stream), "swe_batched_step_static")


def swe_batched_retake(p: swe_params, patches: int, items: int, nitems: int, tasks: int,
                       plain: int, nplain: int, nsub: int, pool_in: int, pool_out: int,
                       pool_work: int, pool_elems: int, pool_b: int, dt_group: int,
                       smax_patch: int, status: int, queue: int, sched: swe_schedule,
                       retake: int, ngroups: int, stream: int = 0,
                       group_status: int = 0) -> None:
    _check(lib().swe_batched_retake(ctypes.byref(p), patches, items, nitems, tasks, plain,
                                    nplain, nsub, pool_in, pool_out, pool_work, pool_elems,
                                    pool_b, dt_group, smax_patch, status, group_status, queue,
                                    ctypes.byref(sched), retake, ngroups, stream),
           "swe_batched_retake")
