"""Benchmark of the agent-mechanics step on one MI355X.

Default workload: the 1M-cell tumour (900k cells in a 600 um ball plus 100k scattered
in a 2 mm cube, radii N(8.4, 0.5) clipped to [6, 11], 30 um voxels, FP32 force
arithmetic with Kahan-compensated sums and FP64 integration).  One step = binning,
counting sort, reorder, 27-voxel forces, Adams-Bashforth and walls, all on the device.

Prints one JSON line: throughput in cell-neighbour interactions/s (value) and
cell-steps/s, step latency p50/p99, the roofline of the force kernel measured with HIP
events on the population's stream, and the CPU oracle timed on a bounded sample.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload tumour1m|sph100k|plain1k]
                  [--precision fp32k|fp32|fp64] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "cell-neighbour interactions/s and cell-steps/s at 1M cells; p50/p99 sim latency"

# MI355X published peaks
PEAK_HBM_GBS = 8000.0
PEAK_FP32_VECTOR_TFLOPS = 157.3
PEAK_FP64_VECTOR_TFLOPS = 78.6

# Algorithmic work of the force kernel (a6 + a7), per unit:
#   candidate pair visited in the 27 voxels: dx, dy, dz (3), d2 (1 mul + 2 fma = 5),
#     R (1), R_A (1), R_A^2 (1)                                       -> 11 FLOP
#   interacting pair: sqrt (1), d (1), 1 - d/R (2), c_rep u^2 (2), 1 - d/R_A (2),
#     C a^2 (2), w (1), w/d (1), three products (3), three sums (3)  -> 18 FLOP
#     (+ 9 for the Kahan compensation of the three sums)              -> 27 FLOP
#   cell: Adams-Bashforth 3 x (2 mul + 1 sub + 1 fma) + walls          -> negligible
FLOP_PER_CANDIDATE = 11
FLOP_PER_INTERACTION = {"fp64": 18, "fp32": 18, "fp32k": 27}
# algorithmic HBM bytes per cell of the force kernel: own f64 position and radius
# (24 + 8) + own and neighbour quantised shadow read once each (8 + 8; the prefilter in
# every precision) + for the pair terms the own and neighbour float shadow once each
# (16 + 16, FP32) or the neighbour's f64 position and radius once (32, FP64) + v_prev
# in/out (24 FP32, 48 FP64) + voxel id (4) + new f64 position (24)
FORCE_BYTES_PER_CELL = {"fp64": 24 + 8 + 16 + 32 + 48 + 4 + 24, "fp32": 24 + 8 + 16 + 32 + 24 + 4 + 24,
                        "fp32k": 24 + 8 + 16 + 32 + 24 + 4 + 24}


def tuning_str(t: dict) -> str:
    return ",".join(str(t[k]) for k in ("force_kernel", "block_waves", "unroll", "blocks_per_cu", "list_len"))


def measured_traffic(kernel: str, workload: str, precision: str, tuning: dict):
    """HBM bytes per launch of `kernel` from its committed counter summary, or None when
    there is none, it was taken with another launch configuration, or the kernel source
    has changed since the counters were taken."""
    from paper_2306_11544_amd import rocprof_summary as RS
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel}_{workload}_{precision}.txt")
    if not os.path.exists(path):
        return None
    for b, sha, _, tun in RS.read_traffic(path):
        if sha == RS.source_sha256() and tun == tuning_str(tuning):
            return b
    return None


def measured_counters(kernel: str, workload: str, precision: str, tuning: dict):
    """Issue and pipe utilisation of `kernel` from its committed PMC summary (None when
    there is none, it was taken with another launch configuration, or the kernel source
    has changed since):
      valu_issue_frac  wave64 VALU instructions / issue slots (one per CU per cycle;
                       GRBM_GUI_ACTIVE sums the 8 XCDs' cycles)
      valu_lane_util   active lanes per VALU instruction / 64
      td_busy_frac     texture-data (vector load return) busy cycles / cycles
      mean_waves_per_cu  rocprofv3's MeanOccupancyPerCU (waves resident per CU, averaged
                       over the kernel's run; 32 is the most a CU holds), when profiled"""
    import re
    from paper_2306_11544_amd import rocprof_summary as RS
    path = os.path.join(ROOT, "profiles", f"pmc_{kernel}_{workload}_{precision}.txt")
    if not os.path.exists(path):
        return None
    for text in RS.sections(path):
        sha = re.search(r"source_sha256\(csrc/mech.hip code\): (\w+)", text)
        tun = re.search(r"--tuning (\S+)", text)
        if sha and sha.group(1) == RS.source_sha256() and tun and tun.group(1) == tuning_str(tuning):
            break
    else:
        return None
    v = {m.group(1): float(m.group(2)) for m in re.finditer(r"^(\w+): ([0-9.e+-]+)", text, re.M)}
    cus, xcds = 256, 8
    cycles = v["GRBM_GUI_ACTIVE"] / xcds
    return {"valu_issue_frac": v["SQ_INSTS_VALU"] / (cus * cycles),
            "valu_lane_util": v["SQ_THREAD_CYCLES_VALU"] / (64.0 * v["SQ_ACTIVE_INST_VALU"]),
            "td_busy_frac": v["TD_TD_BUSY_sum"] / (cus * cycles),
            "mean_waves_per_cu": v.get("MeanOccupancyPerCU"),
            "source": os.path.relpath(path, ROOT)}


def copy_calibration(mb: int, stream):
    """A streaming kernel of known traffic (y = -x over mb MiB of float32: reads and
    writes mb MiB) for scaling the HBM counters of a profiled run."""
    import torch
    n = (mb << 20) // 4
    with torch.cuda.stream(stream):
        src = torch.ones(n, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.neg(src, out=dst)
    torch.cuda.synchronize()
    log(f"copy calibration: 3 x neg over {n * 4} bytes")


def copy_bandwidth(stream, mb: int = 1024, reps: int = 5) -> float:
    """Achieved HBM bandwidth of a plain streaming kernel on this GPU (GB/s): y = -x over
    mb MiB of float32 (reads and writes mb MiB each), timed with HIP events on `stream`."""
    import torch
    n = (mb << 20) // 4
    with torch.cuda.stream(stream):
        src = torch.ones(n, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(2):
            torch.neg(src, out=dst)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            torch.neg(src, out=dst)
        e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del src, dst
    return 2.0 * n * 4 / (ms * 1e-3) / 1e9


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def cpu_baseline(pop, precision: str, budget_s: float = 12.0):
    """The oracle as it stands, on the host cores, on whole steps of the same workload."""
    import oracle
    cores = oracle.set_threads(0)
    p = oracle.params_of(pop)
    prec = {"fp64": oracle.FP64, "fp32": oracle.FP32, "fp32k": oracle.FP32_KAHAN}[precision]
    pos, vp = pop.pos, None
    steps, inter, t_total = 0, 0, 0.0
    while t_total < budget_s and steps < pop.steps:
        t0 = time.perf_counter()
        out = oracle.run(p, pos, pop.radius, pop.type, vp, steps=1, precision=prec)
        t_total += time.perf_counter() - t0
        pos, vp = out["pos"], out["vprev"]
        steps += 1
        inter += out["interactions"]
    return {"value": inter / t_total, "unit": "interactions/s", "cores": cores, "kind": "oracle",
            "cell_steps_per_s": pop.n * steps / t_total,
            "sample": f"{pop.name}: first {steps} step(s) of the full population, "
                      f"{precision} oracle, {t_total:.1f} s"}


def bench_batch(args):
    """256 independent spheroids of log-uniform size in [1k, 100k] advanced in one batch
    (FP32, every kernel of a step launched once for all of them from a captured graph),
    against the plain FP64 path that runs the same simulations one population at a time."""
    import torch

    import workloads
    from paper_2306_11544_amd import binding as B

    n_sims = args.sims
    pops = workloads.batch(n_sims, steps=args.steps)
    prec = args.precision or "fp32"
    p = B.make_params((0, 0, 0), (1, 1, 1), c_adh=workloads.C_ADH_2,
                      precision=B.PRECISIONS[prec], flags=B.FORCE_KERNELS[args.force])
    cells = sum(x.n for x in pops)
    vox = sum(B.batch_request_voxels(p, x.lo, x.hi) for x in pops)
    log(f"batch: {n_sims} simulations, {cells} cells, {vox} voxels, {prec}")
    torch.cuda.init()
    tune_info = None
    best = None
    if args.tune:
        from paper_2306_11544_amd import autotune as A
        t0 = time.perf_counter()
        best, rows = A.tune(p, pops, log=log)
        default_ms = next(r["force_ms"] for r in rows if r == dict(r, **A.DEFAULT.as_dict()))
        tune_info = {"chosen": best.as_dict(), "candidates": len(rows),
                     "force_ms_chosen": min(r["force_ms"] for r in rows),
                     "force_ms_default": default_ms, "seconds": time.perf_counter() - t0}
        log(f"autotuner: {tune_info}")
    with B.Batch(p, cells, vox, n_sims) as bt:
        if best is not None:
            bt.set_tuning(best)
        slots = [bt.admit_pop(x, n_steps=-1) for x in pops]
        bt.step(args.warmup)
        B.batch_sync(bt)
        _, i0, _ = bt.stats()
        t0 = time.perf_counter()
        lat = []
        for _ in range(args.steps):
            ts = time.perf_counter()
            bt.step(1)
            B.batch_sync(bt)
            lat.append((time.perf_counter() - ts) * 1e3)
        wall = time.perf_counter() - t0
        _, i1, _ = bt.stats()
        bin_ms, force_ms = bt.profile(5)
        del slots
    # the plain FP64 path: the same simulations, one population at a time, a few steps each
    sample = pops[:: max(1, n_sims // 16)]
    pstep = 20
    t_fp64 = 0.0
    c_fp64 = 0
    for x in sample:
        with B.Population(B.params_of(x, B.MECH_FP64), x.pos, x.radius, x.type) as P:
            P.step(2)
            P.stats()
            ts = time.perf_counter()
            P.step(pstep)
            P.stats()
            t_fp64 += time.perf_counter() - ts
            c_fp64 += x.n * pstep
    out = {
        "metric": "batched cell-steps/s (FP32, one launch per kernel for all simulations)",
        "value": cells * args.steps / wall, "unit": "cell-steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"batch{n_sims}", "simulations": n_sims, "cells": cells,
                   "voxels": vox, "precision": prec,
                   "tuning": best.as_dict() if best is not None else {"force_kernel": args.force}},
        "autotuner": tune_info,
        "interactions_per_s": (i1 - i0) / wall,
        "step_latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99))},
        "phase_ms": {"binning_reorder": bin_ms, "force_update": force_ms},
        "fp64_per_simulation_path": {"cell_steps_per_s": c_fp64 / t_fp64,
                                     "sample": f"{len(sample)} of the simulations, {pstep} steps each"},
        "speedup_vs_fp64_per_simulation": (cells * args.steps / wall) / (c_fp64 / t_fp64),
    }
    print(json.dumps(out), flush=True)


def bench_locality(args):
    """The paper's locality finding on the GPU: force-kernel time when the cells are
    reordered into voxel order every step (the default), every 10 or 100 steps, or never
    (left in the order they were given in, which is spatially random).  Binning runs
    every step in all modes and the trajectories are bitwise the same; only the memory
    access pattern of the force kernel differs."""
    import torch

    import workloads
    from paper_2306_11544_amd import binding as B

    precision = args.precision or {"tumour1m": "fp32k", "sph100k": "fp64",
                                   "plain1k": "fp64"}[args.workload]
    pop = workloads.config(args.workload)
    prm = B.params_of(pop, B.PRECISIONS[precision])
    torch.cuda.init()
    modes = {}
    for every in (1, 10, 100, 0):
        steps = max(args.steps, 100) if every in (1, 0) else max(args.steps, every)
        with B.Population(prm, pop.pos, pop.radius, pop.type) as P:
            P.step(args.warmup)
            P.set_reorder(every)
            bin_ms, force_ms = P.profile(steps)
            _, inter, cand = P.stats()
        name = "never" if every == 0 else str(every)
        modes[name] = {"steps": steps, "binning_ms": bin_ms, "force_ms": force_ms,
                       "step_ms": bin_ms + force_ms}
        log(f"reorder every {name}: {modes[name]}")
    out = {
        "metric": "force-kernel ms per step by reorder interval (locality ablation)",
        "value": modes["never"]["force_ms"] / modes["1"]["force_ms"],
        "unit": "slowdown of the force kernel without reordering",
        "n_gpus": 1, "higher_is_better": False, "data": "synthetic",
        "config": {"workload": pop.name, "cells": pop.n, "precision": precision,
                   "warmup": args.warmup},
        "modes": modes,
    }
    print(json.dumps(out), flush=True)


def bench_grow(args):
    """The paper's experiment proper: a tumour that grows by division, daughters appended
    at the end of the cell arrays.  Left in that order, the cells lose their spatial
    locality as the population grows; reordered into voxel order every step, they keep
    it.  Force-kernel time per step is sampled as the population doubles, both ways (the
    trajectories are bitwise the same)."""
    import torch

    import workloads
    from paper_2306_11544_amd import binding as B

    precision = args.precision or "fp32k"
    n0, steps, every = 500_000, max(args.steps, 200), 25
    # a dense core that grows into its surroundings; p_div doubles it in about 200 steps
    pop = workloads.tumour(n0, seed=31, steps=steps, core_radius=600 * 0.5 ** (1 / 3),
                           half=1000.0)
    p_div = 2.0 ** (1.0 / 200) - 1.0
    prm = B.params_of(pop, B.PRECISIONS[precision])
    torch.cuda.init()
    series = {}
    # reorder every step, or once at the first step and never again (the cells start in
    # voxel order and daughters pile up at the end)
    for mode in (1, 10 ** 9):
        rows = []
        with B.Population(prm, pop.pos, pop.radius, pop.type, max_cells=2 * n0 + 1000) as P:
            P.set_division(p_div, 1234)
            P.set_reorder(mode)
            for k in range(0, steps + 1, every):
                bin_ms, force_ms = P.profile(3)
                rows.append({"step": k, "cells": P.size(), "binning_ms": bin_ms,
                             "force_ms": force_ms})
                log(f"reorder {mode}: {rows[-1]}")
                if k < steps:
                    P.step(every - 3)
        series["every_step" if mode == 1 else "never"] = rows  # never: after the first step
    last = {m: series[m][-1]["force_ms"] for m in series}
    out = {
        "metric": "force-kernel ms per step as a dividing tumour doubles (locality)",
        "value": last["never"] / last["every_step"],
        "unit": "slowdown without reordering, at the end of the run",
        "n_gpus": 1, "higher_is_better": False, "data": "synthetic",
        "config": {"workload": f"growing tumour {n0}", "precision": precision,
                   "p_div": p_div, "steps": steps},
        "series": series,
    }
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="tumour1m")
    ap.add_argument("--precision", default=None)
    ap.add_argument("--profile-steps", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--sims", type=int, default=256, help="batch workload: simulations")
    ap.add_argument("--cells", type=int, default=0,
                    help="tumour workload with this many cells at the 1M-cell tumour's density "
                         "(core and cube scaled by (cells / 1e6)^(1/3)); a scaling study")
    ap.add_argument("--force", default="cells",
                    help="force kernel when not tuned: cells | rows | voxel")
    ap.add_argument("--no-tune", dest="tune", action="store_false",
                    help="skip the autotuner (default configuration or --force)")
    ap.add_argument("--reorder-every", type=int, default=1,
                    help="reorder the cells every K steps (0: never; the locality study)")
    ap.add_argument("--grow", action="store_true",
                    help="run the growing-tumour locality experiment (division, no reorder)")
    ap.add_argument("--locality", action="store_true",
                    help="run the locality ablation (reorder every 1, 10, 100 steps, never)")
    ap.add_argument("--tuning", default="",
                    help="fixed force-kernel configuration K,W,U,G[,L] (kernel flag, waves per "
                         "workgroup, candidates per trip, workgroups per CU, list entries per "
                         "lane); skips the tuner")
    ap.add_argument("--calibrate-copy-mb", type=int, default=0,
                    help="after the run, a streaming copy of this size for counter scaling")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the mechanics step runs on a single MI355X and "
              "has no multi-GPU path (--gpus must be 1)", file=sys.stderr)
        sys.exit(2)
    if args.workload == "batch":
        bench_batch(args)
        return
    if args.locality:
        bench_locality(args)
        return
    if args.grow:
        bench_grow(args)
        return

    import torch

    import workloads
    from paper_2306_11544_amd import binding as B

    precision = args.precision or {"tumour1m": "fp32k", "sph100k": "fp64",
                                   "plain1k": "fp64"}[args.workload]
    if args.cells and args.workload == "tumour1m":
        f = (args.cells / 1e6) ** (1.0 / 3.0)
        pop = workloads.tumour(args.cells, core_radius=600.0 * f, half=1000.0 * f)
    else:
        pop = workloads.config(args.workload)
    prm = B.params_of(pop, B.PRECISIONS[precision], flags=B.FORCE_KERNELS[args.force])
    log(f"workload {pop.name} n={pop.n} precision={precision} steps={args.steps} "
        f"warmup={args.warmup}")

    torch.cuda.init()
    dev = torch.device("cuda:0")
    stream = torch.cuda.Stream(device=dev)
    ws = torch.empty(B.population_workspace_bytes(prm, pop.n), dtype=torch.uint8, device=dev)
    P = B.Population(prm, pop.pos, pop.radius, pop.type, stream=stream.cuda_stream, workspace=ws)
    tune_info = None
    if args.tuning:
        P.set_tuning(B.tuning(*[int(x) for x in args.tuning.split(",")]))
    elif args.tune:
        from paper_2306_11544_amd import autotune as A
        t0 = time.perf_counter()
        best, rows = A.tune(prm, [pop], log=log)
        default_ms = next(r["force_ms"] for r in rows if r == dict(r, **A.DEFAULT.as_dict()))
        P.set_tuning(best)
        tune_info = {"chosen": best.as_dict(), "candidates": len(rows),
                     "force_ms_chosen": min(r["force_ms"] for r in rows),
                     "force_ms_default": default_ms, "seconds": time.perf_counter() - t0}
        log(f"autotuner: {tune_info}")
    if args.reorder_every != 1:
        P.set_reorder(args.reorder_every)
    tuning = P.get_tuning().as_dict()
    kname = {0: "k_force_cells", B.MECH_FLAG_SIMPLE_FORCE: "k_force_rows",
             B.MECH_FLAG_VOXEL_FORCE: "k_force_lds"}[tuning["force_kernel"]]

    P.step(args.warmup)
    torch.cuda.synchronize()

    # timed region: K steps, inputs already resident in HBM
    _, i0, c0 = P.stats()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    P.step(args.steps)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = e0.elapsed_time(e1)
    _, i1, c1 = P.stats()
    elapsed_s = max(gpu_ms / 1e3, 1e-9)
    inter = i1 - i0
    cand = c1 - c0
    value = inter / elapsed_s
    cell_steps = pop.n * args.steps / elapsed_s
    log(f"timed {args.steps} steps: {gpu_ms:.3f} ms (wall {wall * 1e3:.3f} ms)")

    # per-step latency distribution (one event pair per graph launch)
    lat = []
    nlat = min(args.steps, 100)
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(nlat + 1)]
    evs[0].record(stream)
    for k in range(nlat):
        P.step(1)
        evs[k + 1].record(stream)
    torch.cuda.synchronize()
    lat = np.array([evs[k].elapsed_time(evs[k + 1]) for k in range(nlat)])

    # force kernel alone: HIP events around it on the population's stream
    _, ip0, cp0 = P.stats()
    bin_ms, force_ms = P.profile(args.profile_steps)
    _, ip1, cp1 = P.stats()
    per_launch_inter = (ip1 - ip0) / args.profile_steps
    per_launch_cand = (cp1 - cp0) / args.profile_steps
    flops = FLOP_PER_CANDIDATE * per_launch_cand + FLOP_PER_INTERACTION[precision] * per_launch_inter
    achieved_tflops = flops / (force_ms * 1e-3) / 1e12
    peak = PEAK_FP64_VECTOR_TFLOPS if precision == "fp64" else PEAK_FP32_VECTOR_TFLOPS
    force_bytes = FORCE_BYTES_PER_CELL[precision] * pop.n
    force_gbs = force_bytes / (force_ms * 1e-3) / 1e9
    log(f"phases: binning+reorder {bin_ms:.4f} ms, force+update {force_ms:.4f} ms; "
        f"{achieved_tflops:.2f} TFLOP/s, {force_gbs:.1f} GB/s algorithmic")
    P.close()
    if args.calibrate_copy_mb:
        copy_calibration(args.calibrate_copy_mb, stream)
    copy_gbs = copy_bandwidth(stream)
    log(f"streaming copy: {copy_gbs:.0f} GB/s")
    traffic = measured_traffic(kname, pop.name, precision, tuning)
    counters = measured_counters(kname, pop.name, precision, tuning)

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "interactions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": gpu_ms / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32", "fp32k": "f32"}[precision],
        "data": "synthetic",
        "config": {"workload": pop.name, "cells": pop.n, "precision": precision,
                   "voxel_um": pop.voxel, "dt_min": pop.dt,
                   "integration": "f64 two-step Adams-Bashforth", "tuning": tuning,
                   "reorder_every": args.reorder_every},
        "autotuner": tune_info,
        "cell_steps_per_s": cell_steps,
        "candidates_per_s": cand / elapsed_s,
        "step_latency_ms": {"p50": float(np.percentile(lat, 50)),
                            "p99": float(np.percentile(lat, 99))},
        "phase_ms": {"binning_reorder": bin_ms, "force_update": force_ms},
        "roofline": {"bound": "alu", "kernel": kname, "achieved": achieved_tflops,
                     "peak": peak, "unit": "TFLOP/s", "frac": achieved_tflops / peak,
                     "traffic": traffic,
                     "traffic_GBs": None if traffic is None else traffic / (force_ms * 1e-3) / 1e9,
                     "force_ms_per_launch": force_ms,
                     "counters": counters,
                     "hbm_algorithmic_GBs": force_gbs,
                     "hbm_frac": force_gbs / PEAK_HBM_GBS,
                     # the same rates against what a plain streaming copy reaches here
                     "copy_GBs": copy_gbs,
                     "hbm_frac_of_copy": force_gbs / copy_gbs,
                     "traffic_frac_of_copy": None if traffic is None
                     else traffic / (force_ms * 1e-3) / 1e9 / copy_gbs},
    }
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(pop, precision)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
