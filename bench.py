#!/usr/bin/env python3
"""Benchmark of the two-layer shallow-water hot path on one MI355X.

Default workload: the single-level 4096 x 4096 two-layer grid (dx = 100 m,
r = 0.97, reflecting walls, bathymetry -4000..-50 m, seeded Gaussian surfaces),
stepped with the device-resident dt rule.  One benchmark step is one full
time step of that grid: wall ghost cells, x-sweep, y-sweep, CFL bookkeeping.

Prints one JSON line (rank 0, N = 1):
  value        cell updates per second (interior cells x steps / seconds)
  roofline     the dominant kernel's algorithmic bytes per launch over its
               average HIP-event duration, against 8 TB/s
  cpu_baseline the FP64 oracle on the host, single thread, on a bounded sample
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK = 8.0e12          # bytes/s, MI355X
FP64_PEAK = 78.6e12        # flop/s, MI355X vector FP64
BYTES_PER_CELL = 104       # read 6 state fields + bathymetry, write 6 fields (FP64)
METRIC = "FP64 2-layer cell-updates/s at 1 GPU (% HBM roofline); batched vs plain; adjoint/fwd"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--n", type=int, default=4096, help="grid cells per side")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--cpu-steps", type=int, default=2, help="oracle steps of the full grid")
    ap.add_argument("--copy-probe", type=int, default=0,
                    help="only run a plain device copy of this many MiB (counter calibration)")
    ap.add_argument("--y-rows", type=int, default=0)
    ap.add_argument("--x-rows", type=int, default=0)
    return ap.parse_args()


def kernel_source_sha():
    import hashlib
    d = os.path.join(ROOT, "paper_1803_01450_amd", "csrc")
    src = open(os.path.join(d, "mlswe_kernels.hip"), "rb").read() + open(os.path.join(d, "mlswe_device.hpp"), "rb").read()
    return hashlib.sha256(src).hexdigest()


def profiled_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary, or None if the kernel sources changed since it was taken."""
    path = os.path.join(ROOT, "profiles", "sweeps_roofline_grid_4096_hbm_traffic.md")
    if not os.path.exists(path):
        return None
    sha, val = None, None
    for line in open(path):
        if line.startswith("kernel_source_sha256:"):
            sha = line.split(":", 1)[1].strip()
        if line.startswith("traffic_bytes_per_launch k_%s:" % kernel):
            val = float(line.split(":", 1)[1])
    if sha != kernel_source_sha() or val is None:
        return None
    return val


def copy_probe(mib):
    import torch
    n = mib * (1 << 20) // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes_read": n * 8, "copy_probe_bytes_written": n * 8, "launches": 5}))


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(the sharding design is described in the design notes)", file=sys.stderr)
        sys.exit(2)
    if args.copy_probe:
        copy_probe(args.copy_probe)
        return

    import numpy as np
    import torch
    from paper_1803_01450_amd import inputs
    from paper_1803_01450_amd.binding import Solver

    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(3)
    torch.cuda.init()
    stream = torch.cuda.current_stream()
    print("bench: generating %dx%d roofline grid" % (args.n, args.n), file=sys.stderr, flush=True)
    c = inputs.roofline_grid(n=args.n, L=409.6e3 * args.n / 4096)
    n = c["n"]
    S = Solver(stream=stream.cuda_stream, y_rows=args.y_rows, x_rows=args.x_rows)
    p = S.define(n, n, c["dx"], c["dx"], c["r"])
    # inputs go to HBM before the timed region
    Bd = torch.from_numpy(c["B"]).cuda()
    qd = torch.from_numpy(np.ascontiguousarray(c["q"])).cuda()
    S.set_bathymetry(p, Bd)
    S.set_state(p, 0, qd)
    del Bd, qd
    print("bench: warmup %d steps" % args.warmup, file=sys.stderr, flush=True)
    S.advance(args.warmup)
    S.synchronize()
    torch.cuda.synchronize()

    # timed region: exactly K steps, device-resident dt, no host round trips
    print("bench: timing %d steps" % args.steps, file=sys.stderr, flush=True)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    S.advance(args.steps)
    ev1.record(stream)
    S.synchronize()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    wall = t1 - t0
    ev_ms = ev0.elapsed_time(ev1)
    cells = n * n
    rate = cells * args.steps / wall

    # per-kernel durations from HIP events on the same stream (separate pass)
    S.set_kernel_timing(True)
    nk = min(args.steps, 100)
    S.advance(nk)
    ms, launches = S.kernel_times()
    S.set_kernel_timing(False)
    cnt = S.counters(p)
    status = cnt["status"]
    # algorithmic bytes per launch: x-sweep reads 7 and writes 6 doubles for the
    # n x (n + 4) cells it updates (interior rows and the two frame rows on each
    # side); y-sweep reads 7 and writes 6 for the n x n interior cells
    kinds = [("x_sweep", BYTES_PER_CELL * n * (n + 4)), ("y_sweep", BYTES_PER_CELL * n * n)]
    per = []
    for k, (name, byts) in enumerate(kinds):
        avg = ms[k] / max(1, launches[k]) / 1e3
        per.append(dict(kernel=name, avg_ms=avg * 1e3, launches=launches[k], bytes=byts,
                        gbs=byts / avg / 1e9 if avg > 0 else 0.0))
    dom = max(per, key=lambda d: d["avg_ms"])
    achieved = dom["gbs"]
    traffic = profiled_traffic(dom["kernel"]) if n == 4096 else None
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK / 1e9, "unit": "GB/s",
            "frac": round(achieved * 1e9 / HBM_PEAK, 4), "traffic": traffic,
            "kernel": dom["kernel"], "avg_ms": round(dom["avg_ms"], 4),
            "bytes_per_launch": dom["bytes"], "all_kernels": per}

    out = {
        "metric": METRIC, "value": rate, "unit": "cell-updates/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": wall / args.steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "roofline_grid", "cells": cells, "nx": n, "ny": n, "dx_m": c["dx"],
                   "r": c["r"], "levels": 1, "boundaries": "walls"},
        "step_hbm_frac": round(rate * BYTES_PER_CELL / HBM_PEAK, 4),
        "event_ms_per_step": ev_ms / args.steps,
        "roofline": roof,
        "status": status,
    }
    if not args.no_cpu:
        import oracle
        print("bench: oracle CPU baseline (%d steps of the full grid, 1 thread)" % args.cpu_steps,
              file=sys.stderr, flush=True)
        dt = 0.9 * c["dx"] / np.sqrt(9.81 * 4000.0)
        crate, sec = oracle.time_fixed(c["B"], c["q"], c["dx"], c["dx"], args.cpu_steps, dt, r=c["r"])
        out["cpu_baseline"] = {"value": crate, "unit": "cell-updates/s", "cores": 1, "kind": "oracle",
                               "sample": "%d steps of the full %dx%d grid (%.1f s)" % (args.cpu_steps, n, n, sec)}
    S.close()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
