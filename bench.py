#!/usr/bin/env python3
"""Benchmark of the two-layer shallow-water hot path on one MI355X.

Default workload: the single-level 4096 x 4096 two-layer grid (dx = 100 m,
r = 0.97, reflecting walls, bathymetry -4000..-50 m, seeded Gaussian surfaces),
stepped with the device-resident dt rule.  One benchmark step is one full
time step of that grid: wall ghost cells, x-sweep, y-sweep, CFL bookkeeping.

Prints one JSON line (rank 0, N = 1):
  value        cell updates per second (interior cells x steps / seconds)
  roofline     the step's algorithmic bytes (104 B per cell update) over the
               summed average HIP-event durations of the kernels of one
               step, against 8 TB/s
  cpu_baseline the FP64 oracle on the host on a bounded sample: all threads of
               the process's share (value) and one thread
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
# FP64 flops per cell of one sweep on the 4096^2 workload (fused multiply-add
# counted as two, sign changes as none), from the oracle's operation census of
# one step of that grid (python -m oracle.census): x-sweep over the n x (n + 4)
# cells it updates, y-sweep over the n x n interior
FLOPS_PER_CELL = {"x_sweep": 410.30, "y_sweep": 410.15}
METRIC = "FP64 2-layer cell-updates/s at 1 GPU (% HBM roofline); batched vs plain; adjoint/fwd"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--n", type=int, default=4096, help="grid cells per side")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--cpu-steps", type=int, default=2, help="oracle steps of the full grid, one thread")
    ap.add_argument("--cpu-mt-steps", type=int, default=8, help="oracle steps of the full grid, all threads")
    ap.add_argument("--copy-probe", type=int, default=0,
                    help="only run a plain device copy of this many MiB (counter calibration)")
    ap.add_argument("--y-rows", type=int, default=0)
    ap.add_argument("--x-rows", type=int, default=0)
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the batched-vs-plain, AMR and adjoint measurements")
    ap.add_argument("--batch-problems", type=int, default=512)
    ap.add_argument("--batch-steps", type=int, default=300)
    ap.add_argument("--batch-plain-steps", type=int, default=10)
    ap.add_argument("--amr-steps", type=int, default=200)
    ap.add_argument("--amr-plain-steps", type=int, default=20)
    ap.add_argument("--adjoint-steps", type=int, default=400)
    ap.add_argument("--only", choices=("batch", "amr", "adjoint", "shelf", "layers"), default=None,
                    help="run only this extra measurement and print its JSON (for profiling)")
    ap.add_argument("--modes", default="plain,per_patch,batched,graph,reflux,dynrt",
                    help="launch modes of the batch / AMR measurements")
    return ap.parse_args()


def timed_advance(S, steps, every, tau, mode):
    """Seconds of S.advance(...) bracketed by device synchronisation, and the
    interior cell updates (all levels, all problems) it performed."""
    import torch
    before = sum(sum(S.counters(p)["updates"]) for p in range(len(S.shapes)))
    S.synchronize(); torch.cuda.synchronize()
    t0 = time.perf_counter()
    S.advance(steps, every, tau, mode=mode)
    S.synchronize(); torch.cuda.synchronize()
    t1 = time.perf_counter()
    after = sum(sum(S.counters(p)["updates"]) for p in range(len(S.shapes)))
    return t1 - t0, after - before


def phase_breakdown(S, steps, every, tau, mode):
    """A second pass of the same steps with per-phase HIP-event timing (outside
    the timed region: the events add gaps): milliseconds per coarse step of
    each phase, the regrid as host wall time."""
    S.set_kernel_timing(True)
    S.advance(steps, every, tau, mode=mode)
    ph = S.phase_times()
    S.set_kernel_timing(False)
    return {k: round(ms / steps, 4) for k, (ms, n) in ph.items()}


def bench_batch(nprob, steps, stream, modes=("plain", "per_patch", "batched", "graph"), plain_steps=10):
    """The batch of uneven problems (48..512 cells a side, two levels, ratio 2,
    regrid every 10 steps), after two untimed coarse steps (initial dt, first
    regrid, graph capture): one launch per level substep over all problems
    (eager and graph-replayed) timed over `steps` coarse steps (300: the whole
    run); against them, over the first `plain_steps` coarse steps, plain
    launches (per patch, one problem at a time, each with its own Courant
    check) and per-patch launches of the whole group (one Courant check per
    coarse step), with the batched launches timed over the same steps."""
    import numpy as np
    from paper_1803_01450_amd import inputs
    from paper_1803_01450_amd.binding import Solver, PLAIN, BATCHED, GRAPH, PER_PATCH
    sizes = inputs.batch_sizes(nprob)
    probs = [inputs.batch_problem(k, int(n)) for k, n in enumerate(sizes)]
    tau = np.tile([2e-5, 0.0], (nprob, 1))
    out = {}

    def run(name, mode, nsteps, breakdown=False):
        print("bench: batch %d problems, %s, %d coarse steps" % (nprob, name, nsteps), file=sys.stderr, flush=True)
        S = Solver(stream=stream)
        for c in probs:
            p = S.define(c["n"], c["n"], c["dx"], c["dx"], c["r"], (2,))
            S.set_bathymetry(p, np.kron(c["B"], np.ones((2, 2))))
            S.set_state(p, 0, c["q"])
        if mode in (BATCHED, GRAPH):
            S.autotune(None, reps=1)
        S.advance(2, 10, tau, mode=mode)   # initial dt, first regrid, graph capture
        sec, upd = timed_advance(S, nsteps, 10, tau, mode)
        # the multilevel step's rate against the HBM roof at 104 B per cell update
        res = {"seconds": sec, "coarse_steps": nsteps, "cell_updates": upd, "rate": upd / sec,
               "hbm_frac": round(upd / sec * BYTES_PER_CELL / HBM_PEAK, 4)}
        if breakdown:
            out["tuning"] = S.tuning()
            out["phases_ms_per_coarse_step"] = phase_breakdown(S, 20, 10, tau, mode)
        S.close()
        return res

    for name, mode in (("batched", BATCHED), ("graph", GRAPH)):
        if name in modes:
            out[name] = run(name, mode, steps, breakdown=name == "batched")
    short = [m for m in ("plain", "per_patch") if m in modes]
    for name in short:
        out[name] = run(name, PLAIN if name == "plain" else PER_PATCH, plain_steps)
    if short:
        out["batched_first_steps"] = run("batched", BATCHED, plain_steps)
        for name in short:
            out["batched_vs_" + name] = out["batched_first_steps"]["rate"] / out[name]["rate"]
    if "graph" in out and "batched" in out:
        out["graph_vs_batched"] = out["graph"]["rate"] / out["batched"]["rate"]
    out["problems"] = nprob
    out["level0_cells"] = int(sum(int(n) ** 2 for n in sizes))
    return out


# flag thresholds of the three-level shoreline run (levels 0 and 1): from the
# first regrid's ~0.3M finest cells the refined region follows the spreading
# pulse to ~3M finest cells by coarse step 200, ~2.4e9 cell updates in all
AMR_TAU = [2e-7, 4e-7]


def bench_amr(steps, stream, modes=("plain", "batched", "graph", "reflux", "dynrt"), plain_steps=20):
    """Three levels (ratios 2 and 4) over 400 km with shorelines, 16 level-0
    patches of 64^2, regrid every 4 coarse steps, `steps` coarse steps from the
    initial state (200: the whole run), each mode timed over the whole run.
    "plain" (per-patch launches, one problem at a time) is timed over the first
    `plain_steps` coarse steps, with the batched launches timed over the same
    steps beside it for the ratio.  "reflux": batched launches with the mass
    flux correction at coarse-fine edges; "dynrt": batched with time ratios
    chosen per coarse step."""
    import numpy as np
    from paper_1803_01450_amd import inputs
    from paper_1803_01450_amd.binding import Solver, PLAIN, BATCHED, GRAPH
    c = inputs.amr_shoreline()
    tau = [AMR_TAU]
    out = {}

    def run(name, mode, nsteps, breakdown=False):
        print("bench: AMR 3 levels, %s, %d coarse steps" % (name, nsteps), file=sys.stderr, flush=True)
        S = Solver(stream=stream, reflux=name == "reflux", dynamic_rt=name == "dynrt")
        p = S.define(c["n0"], c["n0"], c["dx0"], c["dx0"], c["r"], c["ratios"])
        S.set_bathymetry(p, c["Bf"])
        S.set_patches(p, 0, c["level0_boxes"])
        S.set_state(p, 0, c["q0"])
        sec, upd = timed_advance(S, nsteps, 4, tau, mode)
        fine = [int(b[2]) * int(b[3]) for b in S.patches(p, 2)]
        res = {"seconds": sec, "coarse_steps": nsteps, "cell_updates": upd, "rate": upd / sec,
               "hbm_frac": round(upd / sec * BYTES_PER_CELL / HBM_PEAK, 4),
               "finest_patches": len(fine), "finest_cells": int(sum(fine)),
               "time_ratios": [int(v) for v in S.time_ratios(p)]}
        if breakdown:
            out["phases_ms_per_coarse_step"] = phase_breakdown(S, 50, 4, tau, mode)
        S.close()
        return res

    for name, mode in (("batched", BATCHED), ("graph", GRAPH), ("reflux", BATCHED), ("dynrt", BATCHED)):
        if name in modes:
            out[name] = run(name, mode, steps, breakdown=name == "batched")
    if "plain" in modes:
        out["plain"] = run("plain", PLAIN, plain_steps)
        out["batched_first_steps"] = run("batched", BATCHED, plain_steps)
        out["batched_vs_plain"] = out["batched_first_steps"]["rate"] / out["plain"]["rate"]
    if "reflux" in out and "batched" in out:
        out["reflux_time_ratio"] = out["reflux"]["seconds"] / out["batched"]["seconds"]
    if "dynrt" in out and "batched" in out:
        out["dynrt_time_ratio"] = out["dynrt"]["seconds"] / out["batched"]["seconds"]
    if "graph" in out and "batched" in out:
        out["graph_vs_batched"] = out["graph"]["rate"] / out["batched"]["rate"]
    out["workload"] = "amr_shoreline_3level_256"
    out["tau"] = AMR_TAU
    return out


def bench_shelf(stream, mode_name="batched"):
    """The paper's demonstration (plane wave onto a shelf, Sec. 3; invented
    parameters): the finest grid everywhere against three levels (ratios 2 and
    4, regrid every 4 coarse steps), both run to the same simulated time.
    Reports the AMR run's share of cell updates and of wall time, beside the
    paper's 7.20 % and 9.57 % (a CPU run, context only)."""
    import numpy as np
    from paper_1803_01450_amd import inputs
    from paper_1803_01450_amd.binding import Solver, BATCHED, GRAPH
    mode = {"batched": BATCHED, "graph": GRAPH}[mode_name]
    c = inputs.shelf_wave()
    T = c["T"]

    def uniform():
        S = Solver(stream=stream)
        p = S.define(c["nfx"], c["nfy"], c["dxf"], c["dxf"], c["r"])
        S.set_bathymetry(p, c["Bf"])
        S.set_state(p, 0, c["qf"])
        S.synchronize()
        t0 = time.perf_counter()
        t = 0.0
        while t < T:
            S.advance(25, mode=mode)
            t = S.counters(p)["t"]
        sec = time.perf_counter() - t0
        upd = sum(S.counters(p)["updates"])
        S.close()
        return {"seconds": sec, "t": t, "cell_updates": upd, "cells": c["nfx"] * c["nfy"]}

    def amr():
        S = Solver(stream=stream)
        p = S.define(c["n0x"], c["n0y"], c["dx0"], c["dx0"], c["r"], c["ratios"])
        S.set_bathymetry(p, c["Bf"])
        S.set_state(p, 0, c["q0"])
        S.synchronize()
        t0 = time.perf_counter()
        t = 0.0
        while t < T:
            S.advance(c["regrid_every"], c["regrid_every"], [c["tau"]], mode=mode)
            t = S.counters(p)["t"]
        sec = time.perf_counter() - t0
        cnt = S.counters(p)
        out = {"seconds": sec, "t": t, "cell_updates": sum(cnt["updates"]), "updates_per_level": cnt["updates"],
               "finest_patches": int(len(S.patches(p, 2)))}
        S.close()
        return out

    print("bench: shelf demonstration, uniform and AMR (%s)" % mode_name, file=sys.stderr, flush=True)
    uniform(); amr()  # warm-up (clocks, code objects)
    u, a = uniform(), amr()
    # per unit of simulated time (the runs stop within one call of T)
    uf = (a["cell_updates"] / a["t"]) / (u["cell_updates"] / u["t"])
    tf = (a["seconds"] / a["t"]) / (u["seconds"] / u["t"])
    return {"uniform": u, "amr": a, "update_fraction": uf, "time_fraction": tf,
            "uniform_rate": u["cell_updates"] / u["seconds"], "amr_rate": a["cell_updates"] / a["seconds"],
            "paper_cpu": {"update_fraction": 0.0720, "time_fraction": 0.0957}, "T": T, "mode": mode_name}


def bench_adjoint(nsteps, stream):
    """1024^2 gauge-misfit run (dt frozen, checkpoints every 20 steps): forward
    time against backward time (recomputation plus adjoint steps)."""
    import numpy as np
    import torch
    from paper_1803_01450_amd import inputs
    from paper_1803_01450_amd.binding import Solver
    from paper_1803_01450_amd.adjoint import MisfitProblem
    print("bench: adjoint 1024^2, %d steps" % nsteps, file=sys.stderr, flush=True)
    c = inputs.adjoint_problem(n=1024)
    dt = 0.9 * c["dx"] / np.sqrt(9.81 * 4000.0)
    dts = np.full(nsteps, dt)
    S = Solver(stream=stream)
    p = S.define(1024, 1024, c["dx"], c["dx"], c["r"])
    S.set_bathymetry(p, c["B"])
    tgt = torch.from_numpy(np.ascontiguousarray(c["targets"][: nsteps // c["every"]])).cuda()
    prob = MisfitProblem(S, p, c["eta2"], dts, c["every"], c["gauge"], tgt, ckpt=c["ckpt"])
    e = torch.from_numpy(c["eta1"]).cuda()
    B = torch.from_numpy(c["B"]).cuda()
    prob.forward(e, B)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    loss, ck = prob.forward(e, B)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prob.backward(e, ck)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    S.close()
    return {"forward_s": t1 - t0, "backward_s": t2 - t1, "adjoint_fwd": (t2 - t1) / (t1 - t0),
            "steps": nsteps, "cells": 1024 * 1024, "loss": float(loss.item())}


def bench_layers(stream, M=4, r=2, n=2048, reps=20):
    """The general M-layer refine and coarsen: four layers with a shore, 2048^2
    coarse cells refined to 4096^2 and coarsened back, each launch timed with
    HIP events on the library's stream.  Algorithmic bytes: refine writes 3M
    doubles and reads the fine bathymetry per fine cell and reads 3M + 1
    doubles per coarse cell; coarsen reads 3M doubles per fine cell and writes
    3M per coarse cell."""
    import torch
    from paper_1803_01450_amd import inputs
    from paper_1803_01450_amd.binding import Solver
    print("bench: M-layer refine / coarsen, M %d, %d^2 -> %d^2" % (M, n, r * n), file=sys.stderr, flush=True)
    c = inputs.layered_problem(M, n, n, r)
    S = Solver(stream=stream)
    qc = torch.from_numpy(c["qc"]).cuda()
    Bc = torch.from_numpy(c["Bc"]).cuda()
    Bf = torch.from_numpy(c["Bf"]).cuda()
    qf = torch.empty((3 * M, r * n, r * n), dtype=torch.float64, device="cuda")
    qc2 = torch.empty_like(qc)
    st = torch.cuda.current_stream()

    def timed(fn):
        for _ in range(3):
            fn()
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
        for e0, e1 in evs:
            e0.record(st)
            fn()
            e1.record(st)
        torch.cuda.synchronize()
        return sum(e0.elapsed_time(e1) for e0, e1 in evs) / reps

    ref_ms = timed(lambda: S.refine_layers(qc, Bc, Bf, qf, r))
    crs_ms = timed(lambda: S.coarsen_layers(qf, qc2, r))
    nf, ncell = (r * n) ** 2, n * n
    ref_b = nf * (3 * M + 1) * 8 + ncell * (3 * M + 1) * 8
    crs_b = nf * 3 * M * 8 + ncell * 3 * M * 8
    S.close()
    return {"layers": M, "ratio": r, "coarse_cells": ncell, "fine_cells": nf,
            "refine": {"avg_ms": ref_ms, "bytes": ref_b, "gbs": ref_b / ref_ms / 1e6,
                       "frac": ref_b / (ref_ms * 1e-3) / HBM_PEAK, "fine_cells_per_s": nf / (ref_ms * 1e-3)},
            "coarsen": {"avg_ms": crs_ms, "bytes": crs_b, "gbs": crs_b / crs_ms / 1e6,
                        "frac": crs_b / (crs_ms * 1e-3) / HBM_PEAK}}


# the sources the sweep kernels are compiled from
SWEEP_SOURCES = ("mlswe_kernels.hip", "mlswe_sweeps_fast.hip", "mlswe_sweeps.inc", "mlswe_wave.hpp",
                 "mlswe_device.hpp", "mlswe_kernels.hpp")


def kernel_source_sha():
    import hashlib
    d = os.path.join(ROOT, "paper_1803_01450_amd", "csrc")
    src = b"".join(open(os.path.join(d, f), "rb").read() for f in SWEEP_SOURCES)
    return hashlib.sha256(src).hexdigest()


def profiled_traffic(kernel):
    """HBM bytes per launch of the kernel named `kernel` from the committed
    rocprofv3 counter summary, or None if the kernel sources changed since it
    was taken (or the summary does not cover that kernel)."""
    path = os.path.join(ROOT, "profiles", "sweeps_roofline_grid_4096_hbm_traffic.md")
    if not os.path.exists(path):
        return None
    sha, val = None, None
    for line in open(path):
        if line.startswith("kernel_source_sha256:"):
            sha = line.split(":", 1)[1].strip()
        if line.startswith("traffic_bytes_per_launch %s:" % kernel):
            val = float(line.split(":", 1)[1])
    if sha != kernel_source_sha() or val is None:
        return None
    return val


def sweep_times(S, nk):
    """Total milliseconds and launch counts of the x and y sweeps over nk steps,
    from HIP events recorded on the library's stream."""
    S.set_kernel_timing(True)
    S.advance(nk)
    ms, launches = S.kernel_times()
    S.set_kernel_timing(False)
    return ms, launches


def copy_probe(mib):
    import torch
    n = mib * (1 << 20) // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes_read": n * 8, "copy_probe_bytes_written": n * 8, "launches": 5}))


def host_cpu():
    """(host threads this process may use, capped at the 16 of one GPU's share;
    the CPU model from /proc/cpuinfo; nproc)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return min(16, n), model, n


def cpu_baseline(c, steps1, steps_mt):
    """The oracle timed on the host on full-size steps of the same grid, in the
    paper's two modes (Sec. 3, Table 1: one thread and several): one thread,
    and all threads of this process's share (rows cut into strips stepped as
    boxes, bit-identical results).  The reported value is the all-threads one."""
    import numpy as np
    import oracle
    threads, model, nproc = host_cpu()
    n = c["n"]
    dt = 0.9 * c["dx"] / np.sqrt(9.81 * 4000.0)
    print("bench: oracle CPU baseline, 1 thread, %d steps" % steps1, file=sys.stderr, flush=True)
    r1, s1 = oracle.time_fixed(c["B"], c["q"], c["dx"], c["dx"], steps1, dt, r=c["r"])
    print("bench: oracle CPU baseline, %d threads, %d steps" % (threads, steps_mt), file=sys.stderr, flush=True)
    rm, sm = oracle.time_fixed_mt(c["B"], c["q"], c["dx"], c["dx"], steps_mt, dt, threads, r=c["r"])
    return {"value": rm, "unit": "cell-updates/s", "cores": threads, "kind": "oracle",
            "sample": "%d steps of the full %dx%d grid on %d threads (%.1f s)" % (steps_mt, n, n, threads, sm),
            "single_thread": {"value": r1, "cores": 1,
                              "sample": "%d steps of the full %dx%d grid (%.1f s)" % (steps1, n, n, s1)},
            "cpu_model": model, "nproc": nproc}


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path", file=sys.stderr)
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
    if args.only:
        modes = tuple(args.modes.split(","))
        st = stream.cuda_stream
        if args.only == "batch":
            res = bench_batch(args.batch_problems, args.batch_steps, st, modes, args.batch_plain_steps)
        elif args.only == "amr":
            res = bench_amr(args.amr_steps, st, modes, args.amr_plain_steps)
        elif args.only == "shelf":
            res = bench_shelf(st)
        elif args.only == "layers":
            res = bench_layers(st)
        else:
            res = bench_adjoint(args.adjoint_steps, st)
        print(json.dumps({args.only: res}))
        return
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
    if not (args.x_rows or args.y_rows):
        # the library's autotuner picks tile heights and schedules for this layout
        print("bench: autotune", file=sys.stderr, flush=True)
        S.autotune(None, reps=3)
    tuning = S.tuning()
    print("bench: warmup %d steps" % args.warmup, file=sys.stderr, flush=True)
    S.advance(args.warmup)
    S.synchronize()
    torch.cuda.synchronize()

    # timed region: exactly K steps, device-resident dt; the Courant number is
    # checked on the host once per window of up to 32 steps (the library's
    # deferred check), not after every step
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
    nk = min(args.steps, 100)
    ms, launches = sweep_times(S, nk)
    cnt = S.counters(p)
    status = cnt["status"]

    # the fast build of the sweeps on the same grid (continuing from this state)
    print("bench: fast build, %d steps" % args.steps, file=sys.stderr, flush=True)
    S.set_tuning(fast=1)
    S.advance(args.warmup)
    S.synchronize()
    torch.cuda.synchronize()
    f0 = time.perf_counter()
    S.advance(args.steps)
    S.synchronize()
    torch.cuda.synchronize()
    fwall = time.perf_counter() - f0
    fms, fl = sweep_times(S, nk)
    S.set_tuning(fast=0)
    fast = {"value": cells * args.steps / fwall, "ms_per_step": fwall / args.steps * 1e3,
            "x_sweep_ms": fms[0] / max(1, fl[0]), "y_sweep_ms": fms[1] / max(1, fl[1]),
            "status": S.counters(p)["status"]}
    # algorithmic bytes per launch: x-sweep reads 7 and writes 6 doubles for the
    # n x (n + 4) cells it updates (interior rows and the two frame rows on each
    # side); y-sweep reads 7 and writes 6 for the n x n interior cells
    # The roofline unit is the cell update: one full step of a cell reads its
    # six fields and B once and writes six once (104 B).  A step's kernels are
    # the x- and y-sweep launches (the split scheme moves its intermediate
    # through HBM between them), so the step's algorithmic bytes are charged to
    # the two together: achieved = 104 B x cells / (x + y average durations).
    # Each sweep's own traffic (seven fields read, six written per swept cell)
    # is listed beside it as a per-kernel bandwidth.
    names = ("x_sweep", "y_sweep")
    # kernels launched: one wave per tile (schedule 0) or persistent waves
    launched = {"x_sweep": "k_sweep_x1" if tuning.get("sched_x", 0) == 0 else "k_sweep_x",
                "y_sweep": "k_sweep_y1" if tuning.get("sched_y", 0) == 0 else "k_sweep_y"}
    sweep_bytes = {"x_sweep": BYTES_PER_CELL * n * (n + 4), "y_sweep": BYTES_PER_CELL * n * n}
    per = []
    for k, name in enumerate(names):
        avg = ms[k] / max(1, launches[k]) / 1e3
        per.append(dict(kernel=launched[name], avg_ms=avg * 1e3, launches=launches[k],
                        sweep_bytes=sweep_bytes[name], sweep_gbs=sweep_bytes[name] / avg / 1e9 if avg > 0 else 0.0))
    step_ms = sum(d["avg_ms"] for d in per)
    step_bytes = BYTES_PER_CELL * n * n
    achieved = step_bytes / (step_ms * 1e-3) / 1e9
    traffic = None
    if n == 4096:
        tr = [profiled_traffic(launched[name]) for name in names]
        traffic = None if any(t is None for t in tr) else sum(tr)
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK / 1e9, "unit": "GB/s",
            "frac": round(achieved * 1e9 / HBM_PEAK, 4), "traffic": traffic,
            "kernel": "+".join(launched[nm] for nm in names), "avg_ms": round(step_ms, 4),
            "bytes_per_launch": step_bytes, "per_kernel": per}
    # the same kernels against the FP64 vector peak, with the census flop count
    if n == 4096:
        fl = FLOPS_PER_CELL["x_sweep"] * n * (n + 4) + FLOPS_PER_CELL["y_sweep"] * n * n
        tf = fl / (step_ms * 1e-3) / 1e12
        roof["alu"] = {"bound": "alu", "achieved": round(tf, 3), "peak": FP64_PEAK / 1e12, "unit": "TFLOP/s",
                       "frac": round(tf * 1e12 / FP64_PEAK, 4),
                       "flops_per_cell": FLOPS_PER_CELL["x_sweep"] + FLOPS_PER_CELL["y_sweep"]}

    out = {
        "metric": METRIC, "value": rate, "unit": "cell-updates/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": wall / args.steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "roofline_grid", "cells": cells, "nx": n, "ny": n, "dx_m": c["dx"],
                   "r": c["r"], "levels": 1, "boundaries": "walls"},
        "step_hbm_frac": round(rate * BYTES_PER_CELL / HBM_PEAK, 4),
        "event_ms_per_step": ev_ms / args.steps,
        "roofline": roof,
        "tuning": tuning,
        "status": status,
        "fast": fast,
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(c, args.cpu_steps, args.cpu_mt_steps)
    S.close()
    if not args.no_extras:
        st = stream.cuda_stream
        out["batch"] = bench_batch(args.batch_problems, args.batch_steps, st, plain_steps=args.batch_plain_steps)
        out["amr"] = bench_amr(args.amr_steps, st, plain_steps=args.amr_plain_steps)
        out["adjoint"] = bench_adjoint(args.adjoint_steps, st)
        out["shelf_demo"] = bench_shelf(st)
        out["layers"] = bench_layers(st)
        out["batched_vs_plain"] = out["batch"]["batched_vs_plain"]
        out["adjoint_fwd"] = out["adjoint"]["adjoint_fwd"]
    print(json.dumps(out))


if __name__ == "__main__":
    main()
