#!/usr/bin/env python3
"""Benchmark of the shallow water patch step on one MI355X.

Headline workload: 4096 x 4096 cells, dx = 250 m, tanh continental shelf with
5% seeded roughness and a dry coast, 2 m Gaussian uplift of sigma 30 km,
extrapolation boundaries; FP64 dimensionally split step with MC-limited
corrections and the CFL rule on the device.  One step = one patch_step launch
(the whole split update) plus the CFL reduction that sets the next dt.

Prints one JSON line.  `value` is cell-updates per second over the timed
steps (state resident in HBM).  `roofline` reports the step kernel's
algorithmic HBM bytes per launch over its average launch time measured with
HIP events on the launch stream.  `cpu_baseline` times the reference solver
(test infrastructure, FP64, OpenMP over rows) on a bounded sample of the same
grid on the host cores.  `variants` adds the FP32 surface-deviation path on
the same grid (and, with --batched, the AMR-shaped patch set).

--calib-copy MB runs only a plain device copy of MB megabytes (for scaling
the FETCH_SIZE / WRITE_SIZE counters of a profiler run).
"""
from __future__ import annotations

import argparse
import copy
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
BYTES_PER_CELL = {0: 56, 1: 28}  # FP64: 4 x 8 B read + 3 x 8 B written; FP32-dev: half


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--n", type=int, default=4096, help="grid side")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--batched", action="store_true",
                    help="also time the coupled AMR hierarchy (the 3000-patch AMR set is timed "
                         "by default)")
    ap.add_argument("--no-batched", action="store_true", help="skip the 3000-patch AMR set")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--traffic", type=str, default=None,
                    help="counter record (key = value) with the step kernel's HBM bytes per launch")
    ap.add_argument("--calib-copy", type=float, default=0.0,
                    help="only run a plain device copy of this many MB, 10 times")
    ap.add_argument("--no-precision-study", action="store_true")
    ap.add_argument("--valu", type=str, default=None,
                    help="counter record (key = value) with the step kernel's SQ counters")
    ap.add_argument("--make-valu-record", nargs=2, metavar=("PMC_ROOT", "OUTDIR"), default=None,
                    help="write the VALU counter records from a rocprofv3 --pmc run and exit")
    ap.add_argument("--make-traffic-record", nargs=2, metavar=("PMC_ROOT", "OUT"), default=None,
                    help="write the traffic record from rocprofv3 --pmc runs and exit")
    ap.add_argument("--amr", action="store_true",
                    help="only the coupled three-level AMR hierarchy (one JSON line)")
    ap.add_argument("--serve", type=int, default=0,
                    help="only run the serving stream with this many requests")
    ap.add_argument("--serve-steps", type=int, default=1000)
    ap.add_argument("--serve-requests", type=int, default=1200,
                    help="requests in the serving run of the default bench (the first sixth "
                         "are warm-up)")
    ap.add_argument("--no-serving", action="store_true")
    return ap.parse_args()


def log(msg):
    print(msg, file=sys.stderr, flush=True)


# sources of the single-patch step kernels (k_split, k_unsplit) that the
# counter records describe
STEP_SOURCES = ("swe_common.hpp", "swe_march.hpp", "swe_math.hpp", "swe_step.hip",
                "swe_unsplit.hpp")


def kernel_source_hash() -> str:
    """Hash of the step kernels' HIP sources and compiler flags; a counter
    record is used only while it carries this hash."""
    import hashlib

    from paper_1901_06798_amd.build import HIPFLAGS
    d = os.path.join(ROOT, "paper_1901_06798_amd", "csrc")
    h = hashlib.sha256(" ".join(HIPFLAGS).encode())
    for name in STEP_SOURCES:
        with open(os.path.join(d, name), "rb") as f:
            h.update(name.encode() + f.read())
    return h.hexdigest()[:16]


TRAFFIC_RECORD = os.path.join(ROOT, "profiles", "k_split_f64_shelf4096_traffic.txt")


def measured_traffic(path: str | None):
    """HBM bytes per launch of the FP64 step kernel from the counter record
    (key = value lines), if it was measured on the current kernel sources."""
    path = path or TRAFFIC_RECORD
    if not os.path.exists(path):
        return None
    rec = {}
    with open(path) as f:
        for line in f:
            if "=" in line and not line.lstrip().startswith("#"):
                k, v = line.split("=", 1)
                rec[k.strip()] = v.strip()
    if rec.get("kernel_source_hash") != kernel_source_hash():
        return None
    try:
        return float(rec["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def _pmc_mean(run_dir: str, counter: str, kernel_sub: str, workgroup: int | None = None,
              first_run: bool = False):
    """Mean of a counter over the dispatches of a kernel; `workgroup` keeps
    only dispatches of that workgroup size (the step kernels' retake launches,
    which end at once unless a step is redone, use 256-thread workgroups, the
    steps themselves 64).  first_run: only the kernel's first run of
    dispatches, up to the first dispatch of another swe kernel of that
    workgroup size (a run of bench.py with its variants times some kernels on
    more than one workload, the shelf first)."""
    import csv
    import glob
    rows = []
    for f in glob.glob(os.path.join(run_dir, "**", "*counter_collection.csv"), recursive=True):
        with open(f) as fh:
            for r in csv.DictReader(fh):
                if r["Counter_Name"] == counter and (
                        workgroup is None or int(r["Workgroup_Size"]) == workgroup):
                    rows.append((int(r["Dispatch_Id"]), r["Kernel_Name"], float(r["Counter_Value"])))
    rows.sort()
    vals = []
    for _, name, v in rows:
        if kernel_sub in name:
            vals.append(v)
        elif first_run and vals and "swe::" in name:
            break
    if not vals:
        raise SystemExit(f"no {counter} samples for {kernel_sub} under {run_dir}")
    return sum(vals) / len(vals), len(vals)


def make_traffic_record(root: str, out: str) -> None:
    """Traffic record of the FP64 step kernel from four rocprofv3 --pmc runs
    under `root`: pmc_fetch/, pmc_write/ (bench.py) and calib_fetch/,
    calib_write/ (bench.py --calib-copy 1024).  Each counter is scaled by the
    ratio of the copy kernel's known bytes to what the counter read for it."""
    kern = "k_split<false, false, false>"
    fetch, nf = _pmc_mean(os.path.join(root, "pmc_fetch"), "FETCH_SIZE", kern, STEP_WG)
    write, nw = _pmc_mean(os.path.join(root, "pmc_write"), "WRITE_SIZE", kern, STEP_WG)
    cf, _ = _pmc_mean(os.path.join(root, "calib_fetch"), "FETCH_SIZE", "copyBuffer")
    cw, _ = _pmc_mean(os.path.join(root, "calib_write"), "WRITE_SIZE", "copyBuffer")
    copy_kib = CALIB_BYTES / 1024.0
    sf, sw = copy_kib / cf, copy_kib / cw
    total = (fetch * sf + write * sw) * 1024.0
    lines = [
        "# FP64 split step k_split<false, false, false>, 4096^2 shelf: HBM traffic per launch",
        "# FETCH_SIZE and WRITE_SIZE (KiB per dispatch) scaled by the copy calibration",
        f"kernel_source_hash = {kernel_source_hash()}",
        f"fetch_kib_per_launch = {fetch:.1f}",
        f"write_kib_per_launch = {write:.1f}",
        f"dispatches_fetch = {nf}",
        f"dispatches_write = {nw}",
        f"calibration_copy_bytes = {CALIB_BYTES}",
        f"calib_fetch_kib = {cf:.1f}",
        f"calib_write_kib = {cw:.1f}",
        f"fetch_scale = {sf:.4f}",
        f"write_scale = {sw:.4f}",
        f"hbm_bytes_per_launch = {total:.0f}",
    ]
    with open(out, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))


CALIB_BYTES = 1024000000
STEP_WG = 64  # threads per workgroup of a step launch (its retake launch uses 256)

VALU_RECORD = os.path.join(ROOT, "profiles", "k_split_f64_shelf4096_valu.txt")
# one VALU lane-operation per lane per clock: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz
VALU_PEAK_LANE_OPS = 256 * 4 * 16 * 2.4e9
SQ_COUNTERS = ("SQ_WAVES", "SQ_INSTS_VALU", "SQ_INSTS_SALU", "SQ_ACTIVE_INST_VALU",
               "SQ_WAVE_CYCLES", "SQ_BUSY_CYCLES", "SQ_WAIT_INST_ANY", "GRBM_GUI_ACTIVE")


# (kernel, record, what, pmc run): sq1 runs the headline step alone
# (--no-variants), sq2 with its variants
VALU_KERNELS = (("k_split<false, false, false>", "k_split_f64_shelf4096_valu.txt",
                 "FP64 split step", "sq1"),
                ("k_split<true, false, false>", "k_split_f32dev_shelf4096_valu.txt",
                 "FP32 surface-deviation split step", "sq2"),
                ("k_unsplit<false>", "k_unsplit_f64_shelf4096_valu.txt", "FP64 unsplit step",
                 "sq2"))


def make_valu_record(root: str, outdir: str) -> None:
    """Instruction counters per dispatch of the step kernels from rocprofv3
    --pmc runs under root/sq1 (bench.py --no-variants: the headline step) and
    root/sq2 (bench.py with its variants; counters SQ_COUNTERS), one record
    per kernel in outdir."""
    for kern, fname, what, run in VALU_KERNELS:
        lines = [f"# {what} {kern}, 4096^2 shelf: SQ counters per dispatch",
                 f"kernel_source_hash = {kernel_source_hash()}"]
        try:
            for c in SQ_COUNTERS:
                v, n = _pmc_mean(os.path.join(root, run), c, kern, STEP_WG, first_run=True)
                lines.append(f"{c} = {v:.0f}")
        except SystemExit as e:
            print(f"skipping {kern}: {e}")
            continue
        lines.append(f"dispatches = {n}")
        with open(os.path.join(outdir, fname), "w") as f:
            f.write("\n".join(lines) + "\n")
        print("\n".join(lines))


def measured_valu(kernel_ms: float, path: str | None = None):
    """VALU figures of the FP64 step kernel from the counter record, if it was
    taken on the current kernel sources."""
    path = path or VALU_RECORD
    if not os.path.exists(path):
        return None
    rec = {}
    with open(path) as f:
        for line in f:
            if "=" in line and not line.lstrip().startswith("#"):
                k, v = line.split("=", 1)
                rec[k.strip()] = v.strip()
    if rec.get("kernel_source_hash") != kernel_source_hash():
        return None
    insts = float(rec["SQ_INSTS_VALU"])
    lane_ops = 64.0 * insts / (kernel_ms * 1e-3)
    return {"valu_insts_per_launch": insts, "salu_insts_per_launch": float(rec["SQ_INSTS_SALU"]),
            "waves_per_launch": float(rec["SQ_WAVES"]),
            "lane_ops_per_s": lane_ops, "peak_lane_ops_per_s": VALU_PEAK_LANE_OPS,
            "frac": lane_ops / VALU_PEAK_LANE_OPS,
            "lane_ops_per_cell_update": 64.0 * insts / (4096.0 * 4096.0)}


OPCOUNT_SHELF = os.path.join(ROOT, "profiles", "oracle_opcount_shelf4096.txt")
OPCOUNT_ACTIVE = os.path.join(ROOT, "profiles", "oracle_opcount_active4096.txt")
# FP64 vector peak of the MI355X as published (256 CUs x 4 SIMDs x 16 lanes x
# 2.4 GHz x 2, an FMA counted as two operations); the step is built without
# contraction (every product and sum rounds as written, as in the reference
# solver), so its ceiling is half of this: one operation per lane per clock
FP64_PEAK_TFLOPS = 78.6
FP64_NO_FMA_TFLOPS = 256 * 4 * 16 * 2.4e9 / 1e12


def _record(path: str) -> dict:
    rec = {}
    if os.path.exists(path):
        with open(path) as f:
            for line in f:
                if "=" in line and not line.lstrip().startswith("#"):
                    k, v = line.split("=", 1)
                    rec[k.strip()] = v.strip()
    return rec


def alu_roofline(kernel_ms: float, record: str, cells: int):
    """Algorithmic FP64 operations of the step (the oracle's count per cell
    update on this workload times the cells) over the launch time."""
    rec = _record(record)
    if "flops_per_cell_update" not in rec:
        return None
    per = float(rec["flops_per_cell_update"])
    tf = per * cells / (kernel_ms * 1e-3) / 1e12
    return {"achieved": tf, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": tf / FP64_PEAK_TFLOPS, "frac_of_no_fma_peak": tf / FP64_NO_FMA_TFLOPS,
            "flops_per_cell_update": per,
            "div_per_cell_update": float(rec.get("div_per_cell_update", "nan")),
            "sqrt_per_cell_update": float(rec.get("sqrt_per_cell_update", "nan")),
            "record": os.path.relpath(record, ROOT)}


def roofline(r64: dict, traffic, valu_path, opcount: str, cells: int) -> dict:
    """Roofline of the headline kernel.  Both bounds are computed: HBM
    (algorithmic bytes per launch over the launch time, against 8 TB/s) and
    ALU (algorithmic FP64 operations per launch, against the FP64 vector
    peak); `bound` names the one the SQ counters say binds: VALU busy time
    above the HBM fraction means the instruction stream, not memory, sets the
    time."""
    kms = r64["kernel_ms_avg"]
    hbm = {"achieved": r64["achieved_gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": r64["achieved_gbs"] / HBM_PEAK_GBS, "alg_bytes_per_launch": r64["alg_bytes"],
           "traffic": traffic,
           "traffic_gbs": traffic / (kms * 1e-3) / 1e9 if traffic else None}
    alu = alu_roofline(kms, opcount, cells)
    valu = measured_valu(kms, valu_path)
    busy = valu["frac"] if valu else None
    bound = "alu" if (alu is not None and busy is not None and busy > hbm["frac"]) else "hbm"
    top = alu if bound == "alu" else hbm
    return {"bound": bound, "achieved": top["achieved"], "peak": top["peak"],
            "unit": top["unit"], "frac": top["frac"], "traffic": traffic,
            "kernel": "swe::k_split<false, false, false>", "kernel_ms_avg": kms,
            "kernel_ms_p50": r64["kernel_ms_p50"], "kernel_ms_p99": r64["kernel_ms_p99"],
            "valu_busy_frac": busy, "hbm": hbm, "alu": alu,
            "why": "VALU busy fraction (SQ counters) above the HBM fraction: the kernel is "
                   "bound by its instruction stream" if bound == "alu" else
                   "no current VALU record, or memory is the larger fraction"}


def edge_stats(h, hu, hv, b, drytol: float = 1e-3, h_fp64: float = 1.0, lanes: int = 64,
               out_cols: int = 60):
    """Share of x-edges between interior cells that are quiet (both cells wet,
    at rest, surface jump (h_R - h_L) + (b_R - b_L) exactly 0), share of
    (row, 64-lane strip) groups whose edges are all quiet (those skip the
    Riemann solve), and share of edges with a cell at or below h_fp64."""
    hL, hR = h[:, :-1], h[:, 1:]
    wet = (hL > drytol) & (hR > drytol)
    rest = (hu[:, :-1] == 0) & (hu[:, 1:] == 0) & (hv[:, :-1] == 0) & (hv[:, 1:] == 0)
    quiet = wet & rest & (((hR - hL) + (b[:, 1:] - b[:, :-1])) == 0.0)
    ny, ne = quiet.shape
    groups = []
    for c0 in range(0, ne, out_cols):
        groups.append(quiet[:, c0: c0 + lanes].all(axis=1))
    strip_rows = np.concatenate(groups)
    shallow = (hL <= h_fp64) | (hR <= h_fp64)
    return {"quiet_edge_frac": float(quiet.mean()),
            "quiet_strip_row_frac": float(strip_rows.mean()),
            "fp64_island_edge_frac": float(shallow.mean())}


def calib_copy(mb: float) -> None:
    import torch
    n = int(mb * 1e6 / 8)
    a = torch.ones(n, dtype=torch.float64, device="cuda:0")
    b = torch.empty_like(a)
    for _ in range(10):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"calib_copy_bytes_read": 8 * n, "calib_copy_bytes_written": 8 * n,
                      "launches": 10}), flush=True)


def copy_sanity(mb: float = 1024.0, reps: int = 10) -> dict:
    """A plain device copy (torch copy_, read + write) timed with HIP events:
    the bandwidth a streaming kernel reaches on this GPU, beside the peak."""
    import torch
    n = int(mb * 1e6 / 8)
    a = torch.ones(n, dtype=torch.float64, device="cuda:0")
    b = torch.empty_like(a)
    b.copy_(a)
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(reps):
        b.copy_(a)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    gbs = 16.0 * n / (ms * 1e-3) / 1e9
    del a, b
    torch.cuda.empty_cache()
    return {"bytes_per_copy": 16 * n, "ms": ms, "gbs": gbs, "frac": gbs / HBM_PEAK_GBS}


def _host_cpu() -> dict:
    model = ""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cpu": model, "nproc": os.cpu_count(), "affinity": len(os.sched_getaffinity(0))}


def cpu_baseline(pb, seconds: float, single_seconds: float = 8.0):
    """Reference solver on the same grid for a bounded number of steps, with
    its OpenMP threads (the machine's CPU share), then on one thread."""
    import oracle as O
    O.lib()
    threads = O.get_threads()
    P = O.params()
    q, b = O.new_state(pb.h, pb.hu, pb.hv, pb.b)
    g = O.grid(pb.mx, pb.my, pb.dx, pb.dy, pb.bc)
    O.ghost_fill_b(g, b)
    O.ghost_fill(g, q)
    sm = O.speed_scan(P, g, q, b)
    dt = P.cfl_desired / max(sm[0] / g.dx, sm[1] / g.dy)
    steps = 0
    t0 = time.perf_counter()
    while True:
        O.run(P, g, q, b, 1, dt0=dt)
        steps += 1
        el = time.perf_counter() - t0
        if el >= seconds or steps >= 50:
            break
    cups = pb.mx * pb.my * steps / el
    out = {"value": cups, "unit": "cell-updates/s", "cores": threads, "kind": "oracle",
           "sample": f"{steps} FP64 split steps of the {pb.mx}x{pb.my} grid "
                     f"({el:.1f} s, {threads} OpenMP threads)"}
    O.set_threads(1)
    try:
        s1 = 0
        t0 = time.perf_counter()
        while True:
            O.run(P, g, q, b, 1, dt0=dt)
            s1 += 1
            el1 = time.perf_counter() - t0
            if el1 >= single_seconds or s1 >= 5:
                break
    finally:
        O.set_threads(threads)
    out["single_thread"] = {"value": pb.mx * pb.my * s1 / el1, "unit": "cell-updates/s",
                            "sample": f"{s1} steps of the same grid ({el1:.1f} s, 1 thread)"}
    out["host"] = _host_cpu()
    return out


def time_patch(pb, params, steps: int, warmup: int, ordered: bool = True, sphere: bool = False):
    """Time `steps` steps of one patch; kernel time from HIP events around each
    step launch on the launch stream (the step ends with the CFL rule in its
    last wave; the sort of the heaviest-first order, when due, and the gated
    retake run after the bracket, inside the timed loop).  sphere: a
    latitude-longitude patch (SphereSolver)."""
    import torch

    from paper_1901_06798_amd import _lib as L
    from paper_1901_06798_amd.solver import PatchSolver
    from paper_1901_06798_amd.sphere import SphereSolver

    if sphere:
        s = SphereSolver(pb, params, "cuda:0", ordered=ordered)
    else:
        s = PatchSolver(pb, params, "cuda:0", ordered=ordered)
    s.initial_dt()
    for _ in range(warmup):
        s.enqueue_step()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    ev0 = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    ev1 = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    start.record(stream)
    for k in range(steps):
        qi, qo = s.q[s.cur].data_ptr(), s.q[1 - s.cur].data_ptr()
        # the step, whose last wave applies the CFL rule (next dt, retake flag)
        ev0[k].record(stream)
        s.launch_step_cfl(qi, qo, stream.cuda_stream)
        ev1[k].record(stream)
        s.after_step(stream.cuda_stream)
        # up to two gated redos, which end at once unless the step went above cfl_max
        s.launch_retake_cfl(qi, qo, stream.cuda_stream, last=0)
        s.launch_retake_cfl(qi, qo, stream.cuda_stream, last=1)
        s.cur ^= 1
    end.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    total_ms = start.elapsed_time(end)
    kern_ms = np.array([a.elapsed_time(b) for a, b in zip(ev0, ev1)])
    flags, clamps = s.flags()
    cells = pb.mx * pb.my
    nbytes = BYTES_PER_CELL[int(params.precision)] * cells
    kavg = float(kern_ms.mean())
    return {"solver": s, "total_ms": total_ms, "wall_s": wall, "ms_per_step": total_ms / steps,
            "cups": cells * steps / (total_ms * 1e-3), "kernel_ms_avg": kavg,
            "kernel_ms_p50": float(np.percentile(kern_ms, 50)),
            "kernel_ms_p99": float(np.percentile(kern_ms, 99)), "alg_bytes": nbytes,
            "achieved_gbs": nbytes / (kavg * 1e-3) / 1e9, "flags": flags, "clamps": clamps}


def time_batched(precision: int, steps: int = 10):
    import torch

    from paper_1901_06798_amd import _lib as L
    from paper_1901_06798_amd import workloads as W
    from paper_1901_06798_amd.batched import BatchedSolver

    specs, probs = W.amr_patch_set()
    trefs = [s.tref for s in specs]
    bs = BatchedSolver(probs, L.params(precision=precision), trefs=trefs,
                       sched=L.schedule(seg=64, waves_per_group=4))
    bs.initial_dt()
    # schedule from the autotuner (timed on this patch set; no cache, so the
    # choice is made on the machine that runs the bench)
    from paper_1901_06798_amd.autotune import _sched_dict, tune
    best = tune(bs, use_cache=False)
    tuned = {"schedule": _sched_dict(best), "candidates": len(bs.tune_results),
             "best_ms": bs.tune_results[0][0], "worst_ms": bs.tune_results[-1][0]}
    bs.run(2)
    bs.capture(2)
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record()
    for _ in range(steps // 2):
        bs.replay()
    t1.record()
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1) / (2 * (steps // 2))
    upd = bs.cells()
    nbytes = BYTES_PER_CELL[precision] * upd
    return {"patches": len(probs), "cell_updates_per_coarse_step": upd,
            "ms_per_coarse_step": ms, "cups": upd / (ms * 1e-3),
            "hbm_gbs_alg": nbytes / (ms * 1e-3) / 1e9,
            "hbm_frac": nbytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "flags": bs.flags()[0], "autotune": tuned,
            "workload": "AMR patch set: 3000 patches (200/800/2000 on levels 1-3, sides "
                        "U{16..96}, seed 3), ratios 4 and 4, 1/4/16 substeps per coarse step, "
                        "one persistent launch per coarse step, graph replay"}


def batched_precision(coarse_steps: int = 10) -> dict:
    """Surface error of the batched FP32 surface-deviation step against the
    batched FP64 step on the AMR patch set (3000 patches, three levels,
    1/4/16 substeps), both with the FP64 run's step sizes; max over cells wet
    (h > 1e-2 m) in both runs."""
    import torch

    from paper_1901_06798_amd import _lib as L
    from paper_1901_06798_amd import workloads as W
    from paper_1901_06798_amd.batched import BatchedSolver

    specs, probs = W.amr_patch_set()
    trefs = [s.tref for s in specs]
    b64 = BatchedSolver(probs, L.params(), trefs=trefs)
    b32 = BatchedSolver(probs, L.params(precision=L.F32_DEV), trefs=trefs)
    b64.initial_dt()
    dts = torch.zeros(coarse_steps, dtype=torch.float64, device=b64.dev)
    for k in range(coarse_steps):
        dts[k].copy_(b64.dt[0])
        b64.enqueue_step(retake=False)
        b32.enqueue_step(cfl=False, dt_ptr=dts.data_ptr() + 8 * k)
        b32.smax.zero_()
    torch.cuda.synchronize()
    worst, worst_deep, wet_cells, moved = 0.0, 0.0, 0, 0.0
    for k in range(len(probs)):
        h64 = b64.state(k)[0]
        h32 = b32.state(k)[0]
        e64, e32 = b64.surface(k), b32.surface(k)
        both = (h64 > 1e-2) & (h32 > 1e-2)
        if both.any():
            d = np.abs(e32 - e64)[both]
            worst = max(worst, float(d.max()))
            deep = both & (h64 > 10.0)
            if deep.any():
                worst_deep = max(worst_deep, float(np.abs(e32 - e64)[deep].max()))
            wet_cells += int(both.sum())
            moved = max(moved, float(np.abs(e64[both] - (probs[k].h + probs[k].b)[both]).max()))
    return {"coarse_steps": coarse_steps, "max_surface_err_m": worst,
            "max_err_deep_m": worst_deep, "bar_m": 1e-5, "within_bar": worst <= 1e-5,
            "wet_cells_compared": wet_cells, "largest_surface_change_m": moved,
            "flags_fp64": b64.flags(), "flags_fp32": b32.flags()}


def time_amr(ncoarse: int = 10, dt1: float = 8.0, precision: int = 0):
    """The seeded three-level hierarchy coupled on the device: eager coarse
    steps, then replays of two captured coarse steps."""
    import torch

    from paper_1901_06798_amd import _lib as L
    from paper_1901_06798_amd import workloads as W
    from paper_1901_06798_amd.amr import AmrSolver

    H = W.amr_nested()
    s = AmrSolver(H, L.params(precision=precision))
    s.set_dt(dt1)
    s.run(2)
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record()
    s.run(4)
    t1.record()
    torch.cuda.synchronize()
    eager_ms = t0.elapsed_time(t1) / 4
    s.capture(2)
    t0.record()
    for _ in range(ncoarse // 2):
        s.replay()
    t1.record()
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1) / (2 * (ncoarse // 2))
    upd = s.cells_per_coarse_step()
    npatch = [sum(1 for p in H.patches if p.level == lev) for lev in (1, 2, 3)]
    nfill, navg = list(s.nfill[1:]), list(s.navg)
    # regrid from the current state (flag |eta| > 0.5 m, buffer 2, efficiency
    # 0.7), then eager coarse steps on the new hierarchy
    rects = s.regrid(tol=0.5, buffer=2, efficiency=0.7)
    regrid = {"tol_m": 0.5, "patches_per_level": [len(x) for x in rects],
              "wall_ms": s.last_regrid_ms,
              "cell_updates_per_coarse_step": s.cells_per_coarse_step()}
    torch.cuda.synchronize()
    t0.record()
    s.run(4)
    t1.record()
    torch.cuda.synchronize()
    regrid["ms_per_coarse_step_after"] = t0.elapsed_time(t1) / 4
    regrid["cups_after"] = regrid["cell_updates_per_coarse_step"] / (
        regrid["ms_per_coarse_step_after"] * 1e-3)
    regrid["flags_after"] = s.flags()[0]
    return {"regrid": regrid, "patches_per_level": npatch, "ratio": H.ratio, "level1_cells": H.n1 * H.n1,
            "cell_updates_per_coarse_step": upd, "ms_per_coarse_step": ms,
            "ms_per_coarse_step_eager": eager_ms, "cups": upd / (ms * 1e-3),
            "ghost_fill_cells_per_substep": nfill, "averaged_cells": navg,
            "max_courant": s.courant(), "flags": s.flags()[0],
            "dt_level1_s": dt1, "coarse_steps_timed": 2 * (ncoarse // 2)}


def precision_study(n: int = 2048, steps: int = 2000, every: int = 250):
    """FP32 surface deviation vs FP64 on the walled shelf.  Both runs advance
    in lockstep (FP32 driven by the FP64 step sizes); at every checkpoint the
    surface error on cells wet (h > 1e-2 m) in both runs is reported, split into
    deep water (h > 10 m) and near shore.  Then a free-running FP32 run, the
    mass drift of both, and the lake-at-rest residual of both paths."""
    import torch

    from paper_1901_06798_amd import _lib as L
    from paper_1901_06798_amd import workloads as W
    from paper_1901_06798_amd.solver import PatchSolver

    pb = W.shelf_walls(n=n, dx=1024e3 / n, seed=4, nsteps=steps)
    res = {"grid": [n, n], "steps": steps, "dx": pb.dx}
    s64 = PatchSolver(pb, L.params())
    s32 = PatchSolver(pb, L.params(precision=L.F32_DEV))
    # the floor FP32 storage alone sets: FP64 arithmetic over the same FP32
    # planes, rounded once per step
    s32w = PatchSolver(pb, L.params(precision=L.F32_STORE))
    # conditioning check: FP64 started from the values the FP32 run starts
    # from (bed and surface deviation rounded to FP32), so only the initial
    # rounding differs from the FP64 run
    sea = L.params().sea_level
    b32 = pb.b.astype(np.float32).astype(np.float64)
    eta32 = np.where(pb.h > 0.0, pb.h + pb.b - sea, pb.b - sea).astype(np.float32).astype(np.float64)
    pbc = copy.copy(pb)
    pbc.b = b32
    pbc.h = np.where(pb.h > 0.0, np.maximum(eta32 + sea - b32, 0.0), 0.0)
    s64c = PatchSolver(pbc, L.params())
    m64, m32 = s64.mass(), s32.mass()
    s64.initial_dt()
    dt_log = torch.zeros(steps, dtype=torch.float64, device=s64.dev)
    hist, hist_c, hist_w = [], [], []

    def errors(a64, a32):
        h64, _, _ = a64.state()
        h32, _, _ = a32.state()
        e64, e32 = a64.surface(), a32.surface()
        both = (h32 > 1e-2) & (h64 > 1e-2)
        err = np.abs(e32 - e64)
        deep = both & (h64 > 10.0)
        shore = both & (h64 <= 10.0)
        return {"max_surface_err_m": float(err[both].max()),
                "max_err_deep_m": float(err[deep].max()) if deep.any() else None,
                "max_err_nearshore_m": float(err[shore].max()) if shore.any() else None,
                "wetdry_mismatch_cells": int(((h32 > 1e-3) != (h64 > 1e-3)).sum()),
                "max_abs_surface_m": float(np.abs(e64[h64 > 1e-2]).max())}

    for k0 in range(0, steps, every):
        for k in range(k0, min(k0 + every, steps)):
            dt_log[k].copy_(s64.dt[0])
            s64.enqueue_step(retake=False)
            s32.enqueue_step(dt_log.data_ptr() + 8 * k, cfl=False)
            s32.smax.zero_()
            s64c.enqueue_step(dt_log.data_ptr() + 8 * k, cfl=False)
            s64c.smax.zero_()
            s32w.enqueue_step(dt_log.data_ptr() + 8 * k, cfl=False)
            s32w.smax.zero_()
        torch.cuda.synchronize()
        e = errors(s64, s32)
        e["step"] = min(k0 + every, steps)
        hist.append(e)
        c = errors(s64, s64c)
        c["step"] = e["step"]
        hist_c.append(c)
        w = errors(s64, s32w)
        w["step"] = e["step"]
        hist_w.append(w)
    res["same_dt"] = dict(hist[-1])
    res["same_dt"]["history"] = hist
    res["fp64_from_fp32_rounded_start"] = dict(hist_c[-1])
    res["fp64_from_fp32_rounded_start"]["history"] = hist_c
    res["fp32_storage_fp64_arithmetic"] = dict(hist_w[-1])
    res["fp32_storage_fp64_arithmetic"]["history"] = hist_w
    del s64c, s32w
    res["mass_drift_fp64"] = (s64.mass() - m64) / m64
    res["same_dt"]["mass_drift_fp32"] = (s32.mass() - m32) / m32
    res["flags_fp64"] = s64.flags()
    res["same_dt"]["flags"] = s32.flags()
    del s32
    f32 = PatchSolver(pb, L.params(precision=L.F32_DEV))
    f32.initial_dt()
    f32.run_async(steps)
    torch.cuda.synchronize()
    res["free_running"] = errors(s64, f32)
    res["free_running"]["flags"] = f32.flags()
    del s64, f32
    rest = W.shelf_walls(n=n, dx=1024e3 / n, seed=4, amp=0.0)
    for prec, name in ((L.F64, "lake_at_rest_fp64"), (L.F32_DEV, "lake_at_rest_fp32_dev")):
        s = PatchSolver(rest, L.params(precision=prec))
        s.run_async(200)
        torch.cuda.synchronize()
        h, hu, hv = s.state()
        wet = rest.h > 0
        res[name] = {"steps": 200, "max_abs_surface_m": float(np.abs(s.surface()[wet]).max()),
                     "max_abs_momentum": float(max(np.abs(hu).max(), np.abs(hv).max()))}
        del s
    return res


def serving(nreq: int, warmup: int, steps: int, rate: float = 20.0, budget_gb: float = 200.0,
            max_slots: int = 64, steps_per_round: int = 50):
    """Poisson stream of scenario requests served with continuous batching;
    each request arrives as its seeded parameters and its grid is built on the
    device at admission."""
    from paper_1901_06798_amd import _lib as L
    from paper_1901_06798_amd import workloads as W
    from paper_1901_06798_amd.serve import Scenario, ScenarioServer

    stream = W.request_stream(count=nreq, rate=rate, nsteps=steps)
    reqs = [Scenario(k, t, None, steps, spec=W.scenario_spec(k, n=n, nsteps=steps))
            for k, t, n in stream]
    srv = ScenarioServer(L.params(precision=L.F32_DEV), hbm_budget=int(budget_gb * (1 << 30)),
                         max_slots=max_slots, steps_per_round=steps_per_round)
    # warm the kernels outside the measured stream
    srv.serve([Scenario(-1, 0.0, None, 50, spec=W.scenario_spec(0, n=256, nsteps=50))],
              label="serve warm-up")
    log(f"[bench] serving: {nreq} requests at {rate}/s, budget {budget_gb} GB")
    out = srv.serve(reqs, warmup=warmup, label=f"serve {budget_gb:g} GB")
    done = out.pop("done")
    out.pop("rejected")
    out.pop("cancelled")
    waits = [sc.admitted - sc.arrival for sc in done if sc.rid >= warmup]
    lat = np.array([sc.finished - sc.arrival for sc in done if sc.rid >= warmup])
    out.update({"rate_per_s": rate, "steps_per_request": steps, "warmup_requests": warmup,
                "hbm_budget_gb": budget_gb, "max_slots": max_slots,
                "steps_per_round": steps_per_round,
                "p90_ms": float(np.percentile(lat, 90) * 1e3) if lat.size else None,
                "max_ms": float(lat.max() * 1e3) if lat.size else None,
                "max_queue_wait_ms": float(max(waits) * 1e3) if waits else None,
                "demand_cell_updates_per_s": rate * steps * float(np.mean(
                    [n * n for _, _, n in stream])),
                "flagged_requests": int(sum(1 for sc in done if sc.result.get("status", 0))),
                "sizes": "n ~ U{256..2048}, dx 500 m", "precision": "fp32_dev",
                "sample": f"{nreq} requests of the Poisson stream (seed 5), the first "
                          f"{warmup} not measured"})
    return out


def serving_pair(nreq: int, steps: int, warmup: int | None = None, small: int = 60) -> dict:
    """The stream with a large HBM budget, then its first `small` requests
    with a budget of about four of the largest grids, which makes requests
    queue for memory."""
    import torch
    out = {"budget_200gb": serving(nreq, nreq // 6 if warmup is None else warmup, steps)}
    torch.cuda.empty_cache()
    small = min(small, nreq)
    out["budget_0.5gb"] = serving(small, max(1, small // 6), steps, budget_gb=0.5)
    return out


def main():
    args = parse()
    if args.make_traffic_record:
        make_traffic_record(*args.make_traffic_record)
        return
    if args.make_valu_record:
        make_valu_record(*args.make_valu_record)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the path is "
              f"single-GPU in this build", file=sys.stderr)
        sys.exit(2)
    import torch

    if not torch.cuda.is_available():
        print("no GPU available", file=sys.stderr)
        sys.exit(1)
    if args.calib_copy > 0:
        calib_copy(args.calib_copy)
        return
    if args.amr:
        out = {"amr_coupled_fp64": time_amr()}
        import torch
        torch.cuda.empty_cache()
        out["amr_coupled_fp32_dev"] = time_amr(precision=1)
        print(json.dumps(out), flush=True)
        return
    if args.serve > 0:
        out = serving_pair(args.serve, args.serve_steps)
        out["metric"] = "scenario latency p50/p99 (ms) and cell-updates/s"
        print(json.dumps(out), flush=True)
        return
    from paper_1901_06798_amd import _lib as L
    from paper_1901_06798_amd import workloads as W

    n = args.n
    log(f"[bench] building {n}x{n} shelf workload")
    pb = W.shelf_4096(n=n, dx=250.0 * 4096 / n)
    log("[bench] FP64 split step")
    r64 = time_patch(pb, L.params(), args.steps, args.warmup)
    log(f"[bench] FP64: {r64['ms_per_step']:.3f} ms/step, kernel {r64['kernel_ms_avg']:.3f} ms, "
        f"{r64['cups']:.3e} CUPS, flags={r64['flags']}")
    traffic = measured_traffic(args.traffic)
    log("[bench] plain device copy (sanity line)")
    copy_line = copy_sanity()
    out = {
        "metric": "cell-updates/s + HBM GB/s, FP64 plain vs batched FP32 at \u22641e-5 m error; p99",
        "value": r64["cups"],
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r64["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"shelf_{n}x{n}_dx{pb.dx:g}_fp64_split", "grid": [n, n],
                   "boundary": "extrapolation", "cfl": 0.9, "limiter": "MC"},
        "roofline": roofline(r64, traffic, args.valu, OPCOUNT_SHELF, n * n),
        "hbm_gbs_alg_step": r64["alg_bytes"] / (r64["ms_per_step"] * 1e-3) / 1e9,
        "copy_sanity": copy_line,
        "status_flags": r64["flags"],
        "clamps": r64["clamps"],
    }
    valu = measured_valu(r64["kernel_ms_avg"], args.valu)
    if valu:
        out["valu"] = valu
    st64 = r64["solver"].state()
    out["edges_at_end"] = edge_stats(*st64, pb.b)
    if not args.no_variants:
        log("[bench] FP32 surface-deviation split step")
        h64 = r64["solver"].surface()
        del r64["solver"]
        torch.cuda.empty_cache()
        r32 = time_patch(pb, L.params(precision=L.F32_DEV), args.steps, args.warmup)
        s32 = r32.pop("solver")
        h32 = s32.surface()
        d32 = s32.state()[0]
        wet = (st64[0] > 1e-2) & (d32 > 1e-2)
        del s32
        out["variants"] = {"fp32_dev": {
            "cups": r32["cups"], "ms_per_step": r32["ms_per_step"],
            "kernel_ms_avg": r32["kernel_ms_avg"], "achieved_gbs": r32["achieved_gbs"],
            "frac": r32["achieved_gbs"] / HBM_PEAK_GBS, "alg_bytes_per_launch": r32["alg_bytes"],
            "speedup_vs_fp64": r32["cups"] / r64["cups"], "flags": r32["flags"],
            "free_running_max_surface_diff_m": float(np.abs(h32 - h64)[wet].max()),
            "free_running_wet_cells": int(wet.sum()),
            "free_running_cells_differing": int((h32 != h64)[wet].sum()),
            "fp64_island_edge_frac": edge_stats(d32, *st64[1:], pb.b)["fp64_island_edge_frac"]}}
        log("[bench] FP64 split step, tasks launched in index order")
        torch.cuda.empty_cache()
        ri = time_patch(pb, L.params(), args.steps, args.warmup, ordered=False)
        ri.pop("solver")
        out["variants"]["fp64_index_order"] = {
            "cups": ri["cups"], "ms_per_step": ri["ms_per_step"],
            "kernel_ms_avg": ri["kernel_ms_avg"], "achieved_gbs": ri["achieved_gbs"],
            "speedup_of_heaviest_first": r64["cups"] / ri["cups"]}
        log("[bench] FP64 unsplit step (transverse waves)")
        torch.cuda.empty_cache()
        ru = time_patch(pb, L.params(method=L.UNSPLIT), args.steps, args.warmup)
        ru.pop("solver")
        out["variants"]["unsplit_fp64"] = {
            "cups": ru["cups"], "ms_per_step": ru["ms_per_step"],
            "kernel_ms_avg": ru["kernel_ms_avg"], "achieved_gbs": ru["achieved_gbs"],
            "frac": ru["achieved_gbs"] / HBM_PEAK_GBS, "flags": ru["flags"]}
        log("[bench] FP64 split step on a sea with no quiet edge")
        torch.cuda.empty_cache()
        pa = W.active_sea(n=n, dx=250.0 * 4096 / n)
        ra = time_patch(pa, L.params(), min(args.steps, 200), args.warmup)
        ra.pop("solver")
        out["variants"]["fully_active_fp64"] = {
            "workload": f"active_sea_{n}x{n}: flat -4000 m, every cell wet, seeded noise in the "
                        "surface and both velocities, so no edge is quiet",
            "cups": ra["cups"], "ms_per_step": ra["ms_per_step"], "kernel_ms_avg": ra["kernel_ms_avg"],
            "achieved_gbs": ra["achieved_gbs"], "hbm_frac": ra["achieved_gbs"] / HBM_PEAK_GBS,
            "flags": ra["flags"],
            "alu": alu_roofline(ra["kernel_ms_avg"], OPCOUNT_ACTIVE, n * n)}
        log("[bench] FP32 surface-deviation split step on the same sea")
        torch.cuda.empty_cache()
        rb = time_patch(pa, L.params(precision=L.F32_DEV), min(args.steps, 200), args.warmup)
        rb.pop("solver")
        out["variants"]["fully_active_fp32_dev"] = {
            "workload": out["variants"]["fully_active_fp64"]["workload"],
            "cups": rb["cups"], "ms_per_step": rb["ms_per_step"], "kernel_ms_avg": rb["kernel_ms_avg"],
            "achieved_gbs": rb["achieved_gbs"], "hbm_frac": rb["achieved_gbs"] / HBM_PEAK_GBS,
            "flags": rb["flags"], "speedup_vs_fp64": rb["cups"] / ra["cups"]}
        del pa
        log("[bench] FP64 split step on a latitude-longitude patch")
        torch.cuda.empty_cache()
        # the extent of the paper's transoceanic domain (longitude -240 .. -100,
        # latitude -31 .. 65) in square cells of 140 / n degrees
        d = 140.0 / n
        ny = int(round(96.0 / d))
        ps = W.latlon_basin(n, ny, lon0=-240.0, lat0=-31.0, dlon=d, dlat=d, amp=2.0,
                            sigma_deg=1.0, src=(-217.5, 38.0), bc=(W.BC_EXTRAP,) * 4)
        rs = time_patch(ps, L.params(), args.steps, args.warmup, sphere=True)
        rs.pop("solver")
        out["variants"]["sphere_fp64"] = {
            "workload": f"latlon_basin_{n}x{ny}_{d * 60:.3g}arcmin_lon-240..-100_lat-31..65",
            "cups": rs["cups"], "ms_per_step": rs["ms_per_step"],
            "kernel_ms_avg": rs["kernel_ms_avg"], "achieved_gbs": rs["achieved_gbs"],
            "frac": rs["achieved_gbs"] / HBM_PEAK_GBS, "flags": rs["flags"],
            "kernel": "swe::k_split_sphere<false>"}
        del ps
        if not args.no_batched:
            for prec, name in ((0, "batched_amr_fp64"), (1, "batched_amr_fp32_dev")):
                log(f"[bench] {name}")
                torch.cuda.empty_cache()
                out["variants"][name] = time_batched(prec)
            b64v, b32v = out["variants"]["batched_amr_fp64"], out["variants"]["batched_amr_fp32_dev"]
            b32v["speedup_vs_fp64_batched"] = b32v["cups"] / b64v["cups"]
            log("[bench] batched FP32 vs FP64 surface error (AMR patch set, 10 coarse steps)")
            torch.cuda.empty_cache()
            b32v["surface_error_vs_fp64"] = batched_precision()
        if args.batched:
            log("[bench] coupled AMR hierarchy (three levels, FP64)")
            torch.cuda.empty_cache()
            out["variants"]["amr_coupled_fp64"] = time_amr()
            torch.cuda.empty_cache()
            out["variants"]["amr_coupled_fp32_dev"] = time_amr(precision=1)
        if not args.no_serving:
            torch.cuda.empty_cache()
            out["serving"] = serving_pair(args.serve_requests, args.serve_steps)
        if not args.no_precision_study:
            log("[bench] precision study (2048^2 walled shelf, 2000 steps)")
            torch.cuda.empty_cache()
            out["precision_study"] = precision_study()
    r64.pop("solver", None)
    if not args.no_cpu_baseline:
        log("[bench] timing the reference solver on the host")
        out["cpu_baseline"] = cpu_baseline(pb, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
