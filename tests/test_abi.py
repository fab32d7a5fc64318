"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every function declared in include/swe.h, its structs have the layout the
Python binding assumes, and argument errors are reported before anything is
launched."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "swe.h")


@pytest.fixture(scope="module")
def L():
    from paper_1901_06798_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_1901_06798_amd import build
        build.build()
    return _lib


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(swe_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_entry_points():
    names = declared_functions()
    for n in ("swe_patch_step", "swe_ghost_fill", "swe_speed_scan", "swe_cfl_reduce", "swe_mass",
              "swe_last_error", "swe_version"):
        assert n in names


def test_library_exports_every_declared_symbol(L):
    lib = L.lib()
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    out = subprocess.run(["nm", "-D", "--defined-only", L.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\bT (swe_[a-z_0-9]+)\b", out))
    assert set(declared_functions()) <= exported


def test_struct_layout_matches_header(L, tmp_path):
    src = tmp_path / "layout.c"
    src.write_text(r'''
#include <stdio.h>
#include <stddef.h>
#include "swe.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu %zu\n", sizeof(swe_params), offsetof(swe_params, method),
         offsetof(swe_params, precision), sizeof(swe_patch), offsetof(swe_patch, mx),
         offsetof(swe_patch, bc), offsetof(swe_patch, reserved));
  return 0;
}
''')
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    vals = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True,
                                           check=True).stdout.split()]
    P, T = L.swe_params, L.swe_patch
    assert vals == [ctypes.sizeof(P), P.method.offset, P.precision.offset, ctypes.sizeof(T),
                    T.mx.offset, T.bc.offset, T.reserved.offset]


def test_argument_errors_are_reported_on_the_host(L):
    lib = L.lib()
    p = L.params()
    pt = L.patch(10, 10, 14, 1.0, 1.0)
    fake = ctypes.c_void_p(0x1000)
    assert lib.swe_patch_step(None, ctypes.byref(pt), fake, fake, fake, fake, fake, fake, None) == L.SWE_EINVAL
    assert b"params" in lib.swe_last_error()
    # pitch too small
    bad = L.patch(10, 10, 12, 1.0, 1.0)
    assert lib.swe_patch_step(ctypes.byref(p), ctypes.byref(bad), fake, ctypes.c_void_p(0x9000000),
                              fake, fake, fake, fake, None) == L.SWE_EINVAL
    assert b"pitch" in lib.swe_last_error()
    # aliasing in/out
    assert lib.swe_patch_step(ctypes.byref(p), ctypes.byref(pt), fake, fake, fake, fake, fake,
                              fake, None) == L.SWE_EINVAL
    assert b"overlap" in lib.swe_last_error()
    # unknown enums
    for field, val in (("order", 3), ("method", 7), ("precision", 9)):
        q = L.params()
        setattr(q, field, val)
        assert lib.swe_patch_step(ctypes.byref(q), ctypes.byref(pt), fake,
                                  ctypes.c_void_p(0x9000000), fake, fake, fake, fake,
                                  None) == L.SWE_EINVAL
    # wall with a single cell
    thin = L.patch(1, 10, 8, 1.0, 1.0)
    assert lib.swe_patch_step(ctypes.byref(p), ctypes.byref(thin), fake, ctypes.c_void_p(0x9000000),
                              fake, fake, fake, fake, None) == L.SWE_EINVAL
    with pytest.raises(L.SweError):
        L.swe_patch_step(p, bad, 0x1000, 0x9000000, 0x1000, 0x1000, 0x1000, 0x1000)


def test_patch_tasks_counts_the_strip_tasks(L):
    # strips of 60 updated columns, chunks of 48 rows (ragged ends included)
    assert L.swe_patch_tasks(L.patch(4096, 4096, 4112, 250.0, 250.0)) == 69 * 86
    assert L.swe_patch_tasks(L.patch(70, 100, 80, 1.0, 1.0)) == 2 * 3
    assert L.swe_patch_tasks(L.patch(60, 48, 64, 1.0, 1.0)) == 1
    assert L.swe_patch_tasks(L.patch(61, 49, 80, 1.0, 1.0)) == 4
    assert L.lib().swe_patch_tasks(ctypes.byref(L.patch(10, 10, 12, 1.0, 1.0)), None) == L.SWE_EINVAL
    with pytest.raises(L.SweError):
        L.swe_patch_tasks(L.patch(10, 10, 12, 1.0, 1.0))


def test_launch_shape_sets_the_task_count_and_workspace(L):
    pt = L.patch(4096, 4096, 4112, 250.0, 250.0)
    assert L.swe_patch_tasks(pt, L.launch()) == 69 * 86
    assert L.swe_patch_tasks(pt, L.launch(rows_per_task=32)) == 69 * 128
    assert L.swe_patch_tasks(pt, L.launch(rows_per_task=60, waves_per_block=4)) == 69 * 69
    # a task never holds more rows than the patch has
    assert L.swe_patch_tasks(L.patch(70, 5, 80, 1.0, 1.0), L.launch(rows_per_task=60)) == 2
    assert L.swe_workspace_bytes(pt) == 8 * 69 * 86
    assert L.swe_workspace_bytes(pt, L.launch(rows_per_task=32)) == 8 * 69 * 128
    lib = L.lib()
    for bad in (L.launch(rows_per_task=61), L.launch(rows_per_task=-1),
                L.launch(waves_per_block=3), L.launch(xcd_run=-2)):
        assert lib.swe_patch_tasks(ctypes.byref(pt), ctypes.byref(bad)) == L.SWE_EINVAL
        assert b"launch" in lib.swe_last_error()
        assert lib.swe_workspace_bytes(ctypes.byref(pt), ctypes.byref(bad)) == 0
    assert lib.swe_workspace_bytes(ctypes.byref(L.patch(10, 10, 12, 1.0, 1.0)), None) == 0


def test_sched_step_rejects_a_null_or_short_schedule(L):
    lib = L.lib()
    p = L.params()
    pt = L.patch(100, 100, 104, 1.0, 1.0)  # 2 strips x 3 chunks of 48 rows
    fake = ctypes.c_void_p(0x1000)
    out = ctypes.c_void_p(0x90000000)
    n = L.swe_patch_tasks(pt)
    assert n == 6
    assert lib.swe_patch_step_sched(ctypes.byref(p), ctypes.byref(pt), fake, out, fake, fake,
                                    fake, fake, None, 0, None, None) == L.SWE_EINVAL
    assert b"schedule" in lib.swe_last_error()
    # the buffer must hold 2 n entries for the launch shape it is used with
    assert lib.swe_patch_step_sched(ctypes.byref(p), ctypes.byref(pt), fake, out, fake, fake,
                                    fake, fake, fake, 2 * n - 1, None, None) == L.SWE_EINVAL
    assert b"shorter" in lib.swe_last_error()
    rows32 = L.launch(rows_per_task=32)
    assert lib.swe_patch_step_sched(ctypes.byref(p), ctypes.byref(pt), fake, out, fake, fake,
                                    fake, fake, fake, 2 * n, ctypes.byref(rows32),
                                    None) == L.SWE_EINVAL
    assert lib.swe_patch_order(ctypes.byref(pt), None, 2 * n, None, None) == L.SWE_EINVAL
    assert b"schedule" in lib.swe_last_error()
    assert lib.swe_patch_order(ctypes.byref(pt), fake, 2 * n - 1, None, None) == L.SWE_EINVAL
    assert b"shorter" in lib.swe_last_error()
    bad = L.patch(10, 10, 12, 1.0, 1.0)
    assert lib.swe_patch_order(ctypes.byref(bad), fake, 100, None, None) == L.SWE_EINVAL
    badl = L.launch(waves_per_block=8)
    assert lib.swe_patch_order(ctypes.byref(pt), fake, 100, ctypes.byref(badl),
                               None) == L.SWE_EINVAL


def test_amr_struct_layout_and_argument_errors(L, tmp_path):
    src = tmp_path / "amr_layout.c"
    src.write_text(r'''
#include <stdio.h>
#include <stddef.h>
#include "swe.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu %zu ", sizeof(swe_amr_rect), offsetof(swe_amr_rect, i0),
         offsetof(swe_amr_rect, j0), offsetof(swe_amr_rect, mx), offsetof(swe_amr_rect, my),
         offsetof(swe_amr_rect, pitch), offsetof(swe_amr_rect, reserved));
  printf("%zu %zu %zu %zu %zu %zu %zu %zu %d %d\n", sizeof(swe_amr_fill_op),
         offsetof(swe_amr_fill_op, st), offsetof(swe_amr_fill_op, wx),
         offsetof(swe_amr_fill_op, wy), offsetof(swe_amr_fill_op, kind),
         sizeof(swe_amr_avg_op), offsetof(swe_amr_avg_op, src), offsetof(swe_amr_avg_op, pitch),
         SWE_AMR_COPY, SWE_AMR_COARSE);
  return 0;
}
''')
    exe = tmp_path / "amr_layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    vals = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True,
                                           check=True).stdout.split()]
    from paper_1901_06798_amd import amr
    R = L.AMR_RECT_DTYPE
    assert vals[:7] == [R.itemsize] + [R.fields[k][1] for k in
                                       ("i0", "j0", "mx", "my", "pitch", "reserved")]
    vals = vals[7:]
    assert vals == [amr.FILL_DTYPE.itemsize, amr.FILL_DTYPE.fields["st"][1],
                    amr.FILL_DTYPE.fields["wx"][1], amr.FILL_DTYPE.fields["wy"][1],
                    amr.FILL_DTYPE.fields["kind"][1],
                    amr.AVG_DTYPE.itemsize, amr.AVG_DTYPE.fields["src"][1],
                    amr.AVG_DTYPE.fields["pitch"][1], L.SWE_AMR_COPY, L.SWE_AMR_COARSE]
    lib = L.lib()
    p = L.params()
    fake = ctypes.c_void_p(0x1000)
    other = ctypes.c_void_p(0x2000)
    # known precision; alpha in [0, 1]; distinct fine and coarse planes
    q9 = L.params()
    q9.precision = 9
    assert lib.swe_amr_fill(ctypes.byref(q9), fake, 1, fake, 8, fake, other, other, 8, fake,
                            0.5, None) == L.SWE_EINVAL
    assert lib.swe_amr_fill(ctypes.byref(p), fake, 1, fake, 8, fake, other, other, 8, fake,
                            1.5, None) == L.SWE_EINVAL
    assert lib.swe_amr_fill(ctypes.byref(p), fake, 1, fake, 8, fake, fake, other, 8, fake,
                            0.5, None) == L.SWE_EINVAL
    assert lib.swe_amr_fill(ctypes.byref(p), fake, 0, fake, 8, fake, other, other, 8, fake,
                            0.5, None) == L.SWE_OK
    assert lib.swe_amr_average(ctypes.byref(p), fake, 1, 0, fake, 8, fake, other, 8, fake,
                               None) == L.SWE_EINVAL
    assert lib.swe_amr_average(ctypes.byref(p), fake, 1, 2, fake, 8, fake, fake, 8, fake,
                               None) == L.SWE_EINVAL
    assert lib.swe_amr_average(ctypes.byref(p), None, 3, 2, fake, 8, fake, other, 8, fake,
                               None) == L.SWE_EINVAL
    # swe_amr_init: ratio >= 1, the new planes differ from the sources, the
    # old table and planes given when n_old > 0; nothing new is no work
    third = ctypes.c_void_p(0x3000)

    def init(ratio=2, n_new=1, cells=16, qn=fake, n_old=1, qo=other, qc=third):
        return lib.swe_amr_init(ctypes.byref(p), ratio, fake, n_new, cells, qn, 8, fake, fake,
                                n_old, qo, 8, fake, 1, qc, 8, fake, None)
    assert init(ratio=0) == L.SWE_EINVAL
    assert init(qo=fake) == L.SWE_EINVAL
    assert init(qc=fake) == L.SWE_EINVAL
    assert init(qo=None) == L.SWE_EINVAL
    assert init(n_new=0) == L.SWE_OK
    assert init(cells=0) == L.SWE_OK
    assert init(n_new=70000) == L.SWE_EINVAL
    # swe_amr_plans: ratio >= 1, non-negative counts, every table and output
    # given when there is work; nothing to plan is no work
    def plans(ratio=2, n_fine=1, entries=16, fill=fake, err=fake):
        return lib.swe_amr_plans(fake, n_fine, fake, 1, ratio, entries, fill, fake, fake, fake,
                                 err, None)
    assert plans(ratio=0) == L.SWE_EINVAL
    assert plans(n_fine=-1) == L.SWE_EINVAL
    assert plans(fill=None) == L.SWE_EINVAL
    assert plans(err=None) == L.SWE_EINVAL
    assert plans(n_fine=0) == L.SWE_OK
    assert plans(entries=0) == L.SWE_OK


def test_amr_plans_match_the_hierarchy(L):
    # host plans only (no GPU): every ghost cell of a fine patch listed once,
    # copies where a same-level patch covers it, the level below elsewhere;
    # every coarse cell under a fine patch averaged once
    import numpy as np
    from paper_1901_06798_amd import amr, workloads as W

    class Lay:  # the pool layout a BatchedSolver would make
        def __init__(self, ps):
            self.offs, self.layout, t = [], [], 0
            for p in ps:
                pitch = -(-(p.mx + 4) // 16) * 16
                size = -(-(pitch * (p.my + 4)) // 64) * 64
                self.offs.append(t)
                self.layout.append((pitch, size))
                t += size

    for r in (1, 2, 4):
        H = W.amr_three_levels(r)
        byl = [[p for p in H.patches if p.level == lev] for lev in (1, 2, 3)]
        geo = [amr._Geo(ps, Lay(ps)) for ps in byl]
        for lev in (1, 2):
            f = amr.fill_plan(geo[lev], geo[lev - 1], r)
            nghost = sum((p.mx + 4) * (p.my + 4) - p.mx * p.my for p in byl[lev])
            assert f.size == nghost and np.unique(f["dst"]).size == nghost
            # the two level-2 patches abut (copies across the seam); level 3's do not
            kinds = {L.SWE_AMR_COPY, L.SWE_AMR_COARSE} if lev == 1 else {L.SWE_AMR_COARSE}
            assert set(int(k) for k in np.unique(f["kind"])) == kinds
            a = amr.average_plan(geo[lev], geo[lev - 1], r)
            assert a.size == sum(p.mx * p.my for p in byl[lev]) // (r * r)
            assert np.unique(a["dst"]).size == a.size


def test_sphere_step_argument_errors(L):
    lib = L.lib()
    pt = L.patch(10, 10, 14, 1.0, 1.0)
    fake = ctypes.c_void_p(0x1000)
    out = ctypes.c_void_p(0x9000000)
    metric = ctypes.c_void_p(0x5000)

    def call(p, patch=pt, m=metric):
        return lib.swe_patch_step_sphere(None if p is None else ctypes.byref(p),
                                         ctypes.byref(patch), fake, out, fake, fake, fake, fake,
                                         m, None, 0, None, None)
    assert call(L.params(), m=None) == L.SWE_EINVAL
    assert b"metric" in lib.swe_last_error()
    for kw in ({"precision": L.F32_DEV}, {"method": L.UNSPLIT}):
        assert call(L.params(**kw)) == L.SWE_EINVAL
        assert b"FP64 split" in lib.swe_last_error()
    assert call(None) == L.SWE_EINVAL
    assert call(L.params(), L.patch(10, 10, 12, 1.0, 1.0)) == L.SWE_EINVAL
    assert b"pitch" in lib.swe_last_error()
    with pytest.raises(L.SweError):
        L.swe_patch_step_sphere(L.params(precision=L.F32_DEV), pt, 0x1000, 0x9000000, 0x1000,
                                0x1000, 0x1000, 0x1000, 0x5000)
    # the sphere's retake, first-step speeds and mass: FP64 split only, a
    # metric and the retake flags required
    rt = ctypes.c_void_p(0x7000)

    def retake(p, m=metric, r=rt):
        return lib.swe_patch_retake_sphere(ctypes.byref(p), ctypes.byref(pt), fake, out, fake,
                                           fake, fake, fake, m, r, None)
    assert retake(L.params(), m=None) == L.SWE_EINVAL
    assert retake(L.params(), r=None) == L.SWE_EINVAL
    assert retake(L.params(precision=L.F32_DEV)) == L.SWE_EINVAL
    assert lib.swe_speed_scan_sphere(ctypes.byref(L.params()), fake, 10, 10, fake, fake, None,
                                     fake, None) == L.SWE_EINVAL
    assert lib.swe_speed_scan_sphere(ctypes.byref(L.params(precision=L.F32_DEV)), fake, 10, 10,
                                     fake, fake, metric, fake, None) == L.SWE_EINVAL
    assert lib.swe_speed_scan_sphere(ctypes.byref(L.params()), fake, 0, 10, fake, fake, metric,
                                     fake, None) == L.SWE_EINVAL
    assert lib.swe_mass_sphere(ctypes.byref(L.params()), fake, fake, None, fake,
                               None) == L.SWE_EINVAL
    assert lib.swe_mass_sphere(ctypes.byref(L.params(method=L.UNSPLIT)), fake, fake, metric,
                               fake, None) == L.SWE_EINVAL

    # the step and the retake with the CFL rule fused: dt, flags and counter
    # required; a metric only with the FP64 split step
    cnt = ctypes.c_void_p(0x8000)

    def fused(p, d=fake, r=rt, c=cnt, m=None):
        return lib.swe_patch_step_cfl(ctypes.byref(p), ctypes.byref(pt), fake, out, fake, d,
                                      fake, fake, r, c, m, None, 0, None, None)

    def fused_retake(p, d=fake, r=rt, c=cnt, m=None):
        return lib.swe_patch_retake_cfl(ctypes.byref(p), ctypes.byref(pt), fake, out, fake, d,
                                        fake, fake, r, c, m, 1, None)
    for f in (fused, fused_retake):
        assert f(L.params(), d=None) == L.SWE_EINVAL
        assert f(L.params(), r=None) == L.SWE_EINVAL
        assert f(L.params(), c=None) == L.SWE_EINVAL
        assert f(L.params(precision=L.F32_DEV), m=metric) == L.SWE_EINVAL


def test_sphere_metric_layout():
    from paper_1901_06798_amd import sphere as S
    import numpy as np
    my = 12
    m = S.metric(-30.0, 0.5, my)
    assert m.shape == (2 * my + 9,)
    kap, ln = m[: my + 4], m[my + 4:]
    # capacities telescope: the rows' areas sum to the band's
    d = np.deg2rad(0.5)
    band = np.sin(np.deg2rad(-30.0 + (my + 2) * 0.5)) - np.sin(np.deg2rad(-30.0 - 2 * 0.5))
    assert np.sum(kap) * d == pytest.approx(band, rel=1e-13)
    assert ln[2] == pytest.approx(np.cos(np.deg2rad(-30.0)), rel=1e-15)
    # a wall at ylo mirrors the two ghost rows and edges, nothing else
    w = S.metric(-30.0, 0.5, my, (1, 1, 0, 1))
    assert w[1] == m[2] and w[0] == m[3]
    assert w[my + 4 + 1] == m[my + 4 + 3] and w[my + 4] == m[my + 4 + 4]
    assert np.array_equal(w[2: my + 4], m[2: my + 4]) and np.array_equal(w[my + 6:], m[my + 6:])


def test_sphere_solver_rejects_polar_frames_on_the_host(L):
    # checked before any device work (the solver needs a GPU only after them)
    from paper_1901_06798_amd import workloads as W
    from paper_1901_06798_amd.sphere import SphereSolver
    for lat0, ny in ((89.0, 4), (-89.6, 10), (80.0, 38)):
        pb = W.latlon_basin(8, ny, lat0=lat0, dlon=0.25, dlat=0.25, amp=0.0)
        with pytest.raises(L.SweError, match="pole"):
            SphereSolver(pb, L.params())
    pb = W.latlon_basin(8, 8, lat0=10.0, dlon=0.25, dlat=0.25, amp=0.0)
    with pytest.raises(L.SweError, match="FP64 split"):
        SphereSolver(pb, L.params(precision=L.F32_DEV))
    pb.meta = {}
    with pytest.raises(L.SweError, match="meta"):
        SphereSolver(pb, L.params())


def test_batched_step_pool_checks(L):
    # every call below is rejected on the host before anything is enqueued
    lib = L.lib()
    sched = L.schedule()
    fake = ctypes.c_void_p(0x1000)
    A, B, C = 0x10000000, 0x20000000, 0x30000000

    def call(nitems, nplain, nsub, pin, pout, pwork, elems, p=L.params()):
        v = lambda x: None if x is None else ctypes.c_void_p(x)
        return lib.swe_batched_step(ctypes.byref(p), fake, fake, nitems, fake, fake, nplain,
                                    nsub, v(pin), v(pout), v(pwork), elems, fake, fake, fake,
                                    fake, None, fake, ctypes.byref(sched), None)

    # items (patches with substeps) and per-substep launches need pool_work
    assert call(3, 0, 0, A, B, None, 100) == L.SWE_EINVAL
    assert b"pool_work" in lib.swe_last_error()
    assert call(0, 5, 2, A, B, None, 100) == L.SWE_EINVAL
    assert b"pool_work" in lib.swe_last_error()
    # overlapping byte ranges are refused, not only equal pointers: 100 FP64
    # elements are 800 bytes, 100 FP32 elements 400
    assert call(3, 0, 0, A, A + 792, C, 100) == L.SWE_EINVAL
    assert b"overlap" in lib.swe_last_error()
    assert call(3, 0, 0, A, B, B + 8, 100) == L.SWE_EINVAL
    assert call(3, 0, 0, C - 8, B, C, 100) == L.SWE_EINVAL
    assert call(3, 0, 0, A, A + 396, C, 100, L.params(precision=L.F32_DEV)) == L.SWE_EINVAL
    assert call(3, 0, 0, A, B, C, 0) == L.SWE_EINVAL
    assert b"pool_elems" in lib.swe_last_error()
    with pytest.raises(L.SweError):
        L.swe_batched_step(L.params(), 0x1000, 0x1000, 3, 0x1000, 0x1000, 0, 0, A, B, 0, 100,
                           0x1000, 0x1000, 0x1000, 0x1000, 0x1000, sched)


def test_state_import_export_argument_errors(L):
    lib = L.lib()
    p = L.params()
    fake = ctypes.c_void_p(0x1000)
    assert lib.swe_state_import(ctypes.byref(p), fake, 1, 10, 10, None, fake, 0, 0, fake, fake,
                                None) == L.SWE_EINVAL
    assert lib.swe_state_import(ctypes.byref(p), fake, -1, 10, 10, fake, fake, 0, 0, fake, fake,
                                None) == L.SWE_EINVAL
    assert lib.swe_state_import(ctypes.byref(p), fake, 1, 0, 10, fake, fake, 0, 0, fake, fake,
                                None) == L.SWE_EINVAL
    assert lib.swe_state_import(ctypes.byref(p), fake, 1, 10, 10, fake, fake, 0, -1, fake, fake,
                                None) == L.SWE_EINVAL
    assert b"src_stride" in lib.swe_last_error()
    f32 = L.params(precision=L.F32_DEV)
    assert lib.swe_state_export(ctypes.byref(f32), fake, 1, 10, 10, fake, None, fake, 0, 0,
                                None) == L.SWE_EINVAL
    assert lib.swe_state_export(ctypes.byref(p), fake, 1, 10, 10, fake, None, None, 0, 0,
                                None) == L.SWE_EINVAL
    assert lib.swe_state_export(ctypes.byref(p), fake, 1, 10, 10, fake, None, fake, 0, -2,
                                None) == L.SWE_EINVAL
    # zero patches enqueue nothing
    assert lib.swe_state_import(ctypes.byref(p), fake, 0, 10, 10, fake, fake, 0, 0, fake, fake,
                                None) == L.SWE_OK


def test_static_batched_step_host_checks(L, tmp_path):
    # the static variant's maximum matches the header, and a pool beyond it is
    # refused on the host before any device call
    src = tmp_path / "static_max.c"
    src.write_text('#include <stdio.h>\n#include "swe.h"\n'
                   'int main(void) { printf("%u\\n", SWE_STATIC_WORK_BYTES); return 0; }\n')
    exe = tmp_path / "static_max"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout
    assert int(out) == L.SWE_STATIC_WORK_BYTES
    lib = L.lib()
    p = L.params()
    sched = L.schedule()
    fake = ctypes.c_void_p(0x1000)
    out_pool = ctypes.c_void_p(0x90000000)
    for prec, esz in ((L.F64, 8), (L.F32_DEV, 4)):
        p.precision = prec
        rc = lib.swe_batched_step_static(ctypes.byref(p), fake, fake, 1, fake, None, 0, 0, fake,
                                         out_pool, L.SWE_STATIC_WORK_BYTES // esz + 1, fake, fake,
                                         fake, fake, None, ctypes.byref(sched), None)
        assert rc == L.SWE_EINVAL
        assert b"static substep pool" in lib.swe_last_error()
