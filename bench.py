#!/usr/bin/env python3
"""Benchmark of the shallow water patch step on one MI355X.

Workload (default): 4096 x 4096 cells, dx = 250 m, tanh continental shelf with
5% seeded roughness and a dry coast, 2 m Gaussian uplift of sigma 30 km,
extrapolation boundaries; FP64 dimensionally split step with the MC-limited
corrections and the CFL rule on the device.  One step = one patch_step launch
(the whole split update) plus the CFL reduction that sets the next dt.

Prints one JSON line.  `value` is cell-updates per second over the timed
steps (state resident in HBM).  `roofline` reports the step kernel's
algorithmic HBM bytes per launch over its average launch time measured with
HIP events on the launch stream.  `cpu_baseline` times the reference solver
(test infrastructure, FP64, OpenMP over rows) on a bounded sample of the same
grid on the host cores.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
BYTES_PER_CELL_F64 = 56  # read h, hu, hv, b (4 x 8 B), write h, hu, hv (3 x 8 B)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--n", type=int, default=4096, help="grid side")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--traffic", type=str, default=None,
                    help="JSON file with measured HBM KiB per launch (fetch, write)")
    return ap.parse_args()


def cpu_baseline(pb, seconds: float):
    """Reference solver on the same grid for a bounded number of steps."""
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
    return {"value": cups, "unit": "cell-updates/s", "cores": threads, "kind": "oracle",
            "sample": f"{steps} FP64 split steps of the {pb.mx}x{pb.my} grid "
                      f"({el:.1f} s, {threads} OpenMP threads)"}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the path is "
              f"single-GPU in this build", file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_1901_06798_amd import _lib as L
    from paper_1901_06798_amd import workloads as W
    from paper_1901_06798_amd.solver import PatchSolver

    if not torch.cuda.is_available():
        print("no GPU available", file=sys.stderr)
        sys.exit(1)
    n = args.n
    print(f"[bench] building {n}x{n} shelf workload", file=sys.stderr, flush=True)
    pb = W.shelf_4096(n=n, dx=250.0 * 4096 / n)
    s = PatchSolver(pb, L.params(), "cuda:0")
    s.initial_dt()
    for _ in range(args.warmup):
        s.enqueue_step()
    torch.cuda.synchronize()
    print(f"[bench] warmup {args.warmup} steps done", file=sys.stderr, flush=True)

    stream = torch.cuda.current_stream()
    ev0 = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    ev1 = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    start.record(stream)
    for k in range(args.steps):
        ev0[k].record(stream)
        L.swe_patch_step(s.p, s.pt, s.q[s.cur].data_ptr(), s.q[1 - s.cur].data_ptr(),
                         s.b.data_ptr(), s.dt.data_ptr(), s.smax.data_ptr(),
                         s.status.data_ptr(), stream.cuda_stream)
        ev1[k].record(stream)
        L.swe_cfl_reduce(s.p, s.pt_dev.data_ptr(), 1, 1, s.smax.data_ptr(), s.dt.data_ptr(),
                         s.status.data_ptr(), 0, 0, stream.cuda_stream)
        s.cur ^= 1
    end.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    total_ms = start.elapsed_time(end)
    kern_ms = np.array([a.elapsed_time(b) for a, b in zip(ev0, ev1)])
    flags, clamps = s.flags()
    print(f"[bench] timed {args.steps} steps: {total_ms:.2f} ms (wall {wall * 1e3:.2f} ms), "
          f"flags={flags} clamps={clamps}", file=sys.stderr, flush=True)

    cells = pb.mx * pb.my
    ms_per_step = total_ms / args.steps
    cups = cells * args.steps / (total_ms * 1e-3)
    alg_bytes = BYTES_PER_CELL_F64 * cells
    kavg = float(kern_ms.mean())
    achieved = alg_bytes / (kavg * 1e-3) / 1e9
    traffic = None
    if args.traffic and os.path.exists(args.traffic):
        with open(args.traffic) as f:
            traffic = json.load(f).get("bytes_per_launch")
    out = {
        "metric": "cell-updates/s (FP64 split step, 4096^2 shelf)",
        "value": cups,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"shelf_{n}x{n}_dx{pb.dx:g}_fp64_split", "grid": [n, n],
                   "boundary": "extrapolation", "cfl": 0.9, "limiter": "MC"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "k_split_f64", "kernel_ms_avg": kavg,
                     "kernel_ms_p50": float(np.percentile(kern_ms, 50)),
                     "kernel_ms_p99": float(np.percentile(kern_ms, 99)),
                     "alg_bytes_per_launch": alg_bytes},
        "hbm_gbs_alg_step": cells * BYTES_PER_CELL_F64 / (ms_per_step * 1e-3) / 1e9,
        "status_flags": flags,
        "clamps": clamps,
    }
    if not args.no_cpu_baseline:
        print("[bench] timing the reference solver on the host", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(pb, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
