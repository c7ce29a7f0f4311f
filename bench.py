"""Benchmark of the agent-mechanics step (and the microenvironment solver) on one MI355X.

Headline: the 1M-cell tumour (900k cells in a 600 um ball plus 100k scattered in a 2 mm
cube, radii N(8.4, 0.5) clipped to [6, 11], 30 um voxels) in FP64, the paper's working
precision.  One step = binning, counting sort, reorder, 27-voxel forces, Adams-Bashforth
and walls, all on the device.  `value` is cell-neighbour interactions/s over exactly
--steps timed steps with the state resident in HBM; cell-steps/s and step latency sit
beside it, with the force kernel's roofline measured live (HIP events on the stream it
runs on) and the FP64 oracle timed on the host cores.

Further legs of the same JSON line (each bounded to seconds; --legs selects them):
  fp32k     the same workload with FP32 pair terms and Kahan-compensated sums, and its
            difference from the FP64 run after the same steps
  batch     256 independent spheroids (1k..100k cells) advanced together in FP32 from
            captured graphs, against the plain FP64 path running them one population at
            a time: cell-steps/s, step latency and per-simulation completion p50/p99
  serving   Poisson requests (50/s, 1k..500k cells, 10..1000 steps) admitted into an
            arena sized from a 200 GiB HBM budget: request latency p50/p99, cell-steps/s
  microenv  the microenvironment solver on the paper's 75^3 mesh (one substrate): ms per
            step, voxel updates/s, HBM roofline, and its oracle on the host cores

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload tumour1m|sph100k|plain1k]
                  [--precision fp64|fp32k|fp32] [--legs fp32k,batch,serving,microenv]
                  [--no-cpu-baseline]
  python bench.py --workload batch | --workload microenv | --locality | --grow
                                                            (standalone studies)
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
PEAK_FP32_VECTOR_TFLOPS = 157.3        # packed FP32 (two operations per lane and cycle)
PEAK_FP32_UNPACKED_TFLOPS = 78.6       # what FP32 code compiled without packed-FP32 ops can issue
PEAK_FP64_VECTOR_TFLOPS = 78.6

# Algorithmic work of the force kernel (a6 + a7), per unit, as the method counts it:
#   candidate pair tested (a cell of the 27 surrounding voxels): the difference vector
#     (3), d^2 (5: three products, two sums), R = r_i + r_j (1), R_A (1), R_A^2 (1),
#     the comparisons (1)                                              -> 12 FLOP
#   interacting pair (0 < d < R_A): d (square root), 1 - d/R and its square times c_rep,
#     1 - d/R_A and its square times C[t_i][t_j], w / d, the three products and the
#     three sums, with the square root and the two divisions counted as the several
#     operations they take                                             -> 35 FLOP
#     (+ 12 for the Kahan compensation of the three sums)              -> 47 FLOP
#   cell: Adams-Bashforth and walls                                    -> negligible
# Candidates and interactions are the kernel's exact counters.  A kernel that tests
# fewer candidates for the same pairs (the slab window) is credited only with the
# candidates it tests.
FLOP_PER_CANDIDATE = 12
FLOP_PER_INTERACTION = {"fp64": 35, "fp32": 35, "fp32k": 47}
# algorithmic HBM bytes per cell of the force kernel: own f64 position and radius
# (24 + 8) + own and neighbour quantised shadow read once each (8 + 8; the prefilter in
# every precision) + for the pair terms the own and neighbour float shadow once each
# (16 + 16, FP32) or the neighbour's f64 position and radius once (32, FP64) + v_prev
# in/out (24 FP32, 48 FP64) + voxel id (4) + new f64 position (24)
FORCE_BYTES_PER_CELL = {"fp64": 24 + 8 + 16 + 32 + 48 + 4 + 24, "fp32": 24 + 8 + 16 + 32 + 24 + 4 + 24,
                        "fp32k": 24 + 8 + 16 + 32 + 24 + 4 + 24}
# microenvironment: each of the three solves of a step reads and writes every density
# once (8 + 8 bytes per voxel and substrate); the gradient kernel reads it once and
# writes three gradients (8 + 24)
ENV_BYTES_PER_SOLVE = 16
ENV_BYTES_GRADIENT = 32
ALL_LEGS = ("fp32k", "batch", "serving", "microenv")


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
                       over the kernel's run; 32 is the most a CU holds), when profiled
      valu_insts_per_candidate  wave64 VALU instructions x 64 x lane utilisation per
                       tested candidate (lane-instructions a candidate costs), when the
                       summary records the candidates per launch"""
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
    lane = v["SQ_THREAD_CYCLES_VALU"] / (64.0 * v["SQ_ACTIVE_INST_VALU"])
    out = {"valu_issue_frac": v["SQ_INSTS_VALU"] / (cus * cycles),
           "valu_lane_util": lane,
           "td_busy_frac": v["TD_TD_BUSY_sum"] / (cus * cycles),
           "mean_waves_per_cu": v.get("MeanOccupancyPerCU"),
           "source": os.path.relpath(path, ROOT)}
    if "candidates_per_launch" in v:
        out["valu_insts_per_candidate"] = v["SQ_INSTS_VALU"] * 64.0 * lane / v["candidates_per_launch"]
    return out


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


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def cpu_baseline(pop, precision: str, repeats: int = 5, repeats_1core: int = 3):
    """The oracle as it stands, on the host cores: one whole step of the workload from
    its initial state, timed `repeats` times on all the cores OpenMP is given and
    `repeats_1core` times on one core; the medians are reported."""
    import oracle
    p = oracle.params_of(pop)
    prec = {"fp64": oracle.FP64, "fp32": oracle.FP32, "fp32k": oracle.FP32_KAHAN}[precision]
    cores = oracle.set_threads(0)

    def timed(n_rep):
        ts, inter = [], 0
        for _ in range(n_rep):
            t0 = time.perf_counter()
            out = oracle.run(p, pop.pos, pop.radius, pop.type, None, steps=1, precision=prec)
            ts.append(time.perf_counter() - t0)
            inter = out["interactions"]
        return float(np.median(ts)), inter, ts

    t_all, inter, ts_all = timed(repeats)
    oracle.set_threads(1)
    try:
        t_one, _, ts_one = timed(repeats_1core)
    finally:
        oracle.set_threads(cores)
    return {"value": inter / t_all, "unit": "interactions/s", "cores": cores, "kind": "oracle",
            "cell_steps_per_s": pop.n / t_all,
            "one_core": {"value": inter / t_one, "cell_steps_per_s": pop.n / t_one,
                         "seconds_per_step_median": t_one, "repeats": repeats_1core},
            "seconds_per_step_median": t_all, "repeats_s": ts_all, "cpu_model": cpu_model(),
            "sample": f"{pop.name}: its first step (from the initial state), {precision} oracle, "
                      f"median of {repeats} runs on {cores} threads and of {repeats_1core} on one"}


def external_stream(handle: int):
    import torch
    return torch.cuda.ExternalStream(handle, device="cuda:0")


def measure_population(pop, precision: str, args, tune: bool):
    """Warm-up, exactly args.steps timed steps, per-step latencies and the force kernel's
    roofline for one population in one precision.  Returns (record, positions after
    warmup + steps steps)."""
    import torch

    from paper_2306_11544_amd import binding as B

    prm = B.params_of(pop, B.PRECISIONS[precision], flags=B.FORCE_KERNELS[args.force])
    dev = torch.device("cuda:0")
    stream = torch.cuda.Stream(device=dev)
    ws = torch.empty(B.population_workspace_bytes(prm, pop.n), dtype=torch.uint8, device=dev)
    P = B.Population(prm, pop.pos, pop.radius, pop.type, stream=stream.cuda_stream, workspace=ws)
    tune_info = None
    if args.tuning:
        P.set_tuning(B.tuning(*[int(x) for x in args.tuning.split(",")]))
    elif tune:
        from paper_2306_11544_amd import autotune as A
        t0 = time.perf_counter()
        best, rows = A.tune(prm, [pop], log=None)
        P.set_tuning(best)
        tune_info = {"chosen": best.as_dict(), "candidates": len(rows),
                     "force_ms_chosen": A.chosen_ms(rows, best),
                     "force_ms_default": A.chosen_ms(rows, A.DEFAULT),
                     "seconds": time.perf_counter() - t0}
        log(f"{precision} autotuner: {tune_info}")
    if args.reorder_every != 1:
        P.set_reorder(args.reorder_every)
    tuning = P.get_tuning().as_dict()
    kname = {0: "k_force_cells", B.MECH_FLAG_SIMPLE_FORCE: "k_force_rows",
             B.MECH_FLAG_VOXEL_FORCE: "k_force_lds",
             B.MECH_FLAG_PRUNED_FORCE: "k_force_cells"}[tuning["force_kernel"]]

    P.step(args.warmup)
    torch.cuda.synchronize()
    # timed region: exactly args.steps steps, inputs already resident in HBM
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
    pos_after, _ = P.state()
    elapsed_s = max(gpu_ms / 1e3, 1e-9)
    inter, cand = i1 - i0, c1 - c0
    log(f"{precision}: timed {args.steps} steps: {gpu_ms:.3f} ms (wall {wall * 1e3:.3f} ms)")

    # per-step latency distribution (one event pair per graph launch)
    nlat = max(1, min(args.steps, 100))
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(nlat + 1)]
    evs[0].record(stream)
    for k in range(nlat):
        P.step(1)
        evs[k + 1].record(stream)
    torch.cuda.synchronize()
    lat = np.array([evs[k].elapsed_time(evs[k + 1]) for k in range(nlat)])

    # the force kernel alone: HIP events around each of its launches, on its stream
    _, ip0, cp0 = P.stats()
    bin_ms, force_ms = P.profile(args.profile_steps)
    _, ip1, cp1 = P.stats()
    P.close()
    del ws
    per_inter = (ip1 - ip0) / args.profile_steps
    per_cand = (cp1 - cp0) / args.profile_steps
    flops = FLOP_PER_CANDIDATE * per_cand + FLOP_PER_INTERACTION[precision] * per_inter
    achieved = flops / (force_ms * 1e-3) / 1e12
    peak = PEAK_FP64_VECTOR_TFLOPS if precision == "fp64" else PEAK_FP32_VECTOR_TFLOPS
    force_bytes = FORCE_BYTES_PER_CELL[precision] * pop.n
    force_gbs = force_bytes / (force_ms * 1e-3) / 1e9
    log(f"{precision}: binning+reorder {bin_ms:.4f} ms, force+update {force_ms:.4f} ms; "
        f"{achieved:.2f} TFLOP/s, {force_gbs:.1f} GB/s algorithmic")
    traffic = measured_traffic(kname, pop.name, precision, tuning)
    counters = measured_counters(kname, pop.name, precision, tuning)
    roof = {"bound": "alu", "kernel": kname, "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
            "frac": achieved / peak, "traffic": traffic,
            "flop_model": {"per_candidate": FLOP_PER_CANDIDATE,
                           "per_interaction": FLOP_PER_INTERACTION[precision],
                           "candidates_per_launch": per_cand, "interactions_per_launch": per_inter},
            "force_ms_per_launch": force_ms,
            "traffic_GBs": None if traffic is None else traffic / (force_ms * 1e-3) / 1e9,
            "counters": counters,
            "hbm_algorithmic_GBs": force_gbs, "hbm_frac": force_gbs / PEAK_HBM_GBS}
    if precision != "fp64":
        roof["frac_of_unpacked_fp32"] = achieved / PEAK_FP32_UNPACKED_TFLOPS
    rec = {"value": inter / elapsed_s, "unit": "interactions/s", "steps": args.steps,
           "ms_per_step": gpu_ms / args.steps, "cell_steps_per_s": pop.n * args.steps / elapsed_s,
           "candidates_per_s": cand / elapsed_s,
           "step_latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99))},
           "phase_ms": {"binning_reorder": bin_ms, "force_update": force_ms},
           "tuning": tuning, "autotuner": tune_info, "roofline": roof}
    return rec, pos_after


def leg_batch(args, n_sims=256, steps=20, warmup=3):
    """C4: 256 spheroids advanced together in FP32, against the plain FP64 path that runs
    the same simulations one population at a time (each resident on the device, run
    back to back).  Completion of simulation k: the batch finishes every simulation at
    its last step; the per-simulation path finishes simulation k after the steps of
    simulations 0..k."""
    import torch

    import workloads
    from paper_2306_11544_amd import binding as B

    pops = workloads.batch(n_sims, steps=steps)
    p = B.make_params((0, 0, 0), (1, 1, 1), c_adh=workloads.C_ADH_2, precision=B.MECH_FP32)
    cells = sum(x.n for x in pops)
    vox = sum(B.batch_request_voxels(p, x.lo, x.hi) for x in pops)
    tune_info = None
    best = None
    if args.tune:
        from paper_2306_11544_amd import autotune as A
        t0 = time.perf_counter()
        best, rows = A.tune(p, pops)
        tune_info = {"chosen": best.as_dict(), "candidates": len(rows),
                     "force_ms_chosen": A.chosen_ms(rows, best),
                     "force_ms_default": A.chosen_ms(rows, A.DEFAULT),
                     "seconds": time.perf_counter() - t0}
    with B.Batch(p, cells, vox, n_sims) as bt:
        if best is not None:
            bt.set_tuning(best)
        for x in pops:
            bt.admit_pop(x, n_steps=-1)
        bt.step(warmup)
        bt.sync()
        s = external_stream(bt.stream)
        _, i0, _ = bt.stats()
        evs = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
        evs[0].record(s)
        for k in range(steps):
            bt.step(1)
            evs[k + 1].record(s)
        torch.cuda.synchronize()
        _, i1, _ = bt.stats()
        lat = np.array([evs[k].elapsed_time(evs[k + 1]) for k in range(steps)])
        total_ms = evs[0].elapsed_time(evs[-1])
        bin_ms, force_ms = bt.profile(5)
        tuning = bt.get_tuning().as_dict()
    # the plain FP64 path: one population per simulation, all resident, run one after
    # another for the same steps
    popsP = [B.Population(B.params_of(x, B.MECH_FP64), x.pos, x.radius, x.type) for x in pops]
    try:
        for P in popsP:
            P.step(2)   # first launch captures its graph
        torch.cuda.synchronize()
        t_sim = []
        for P in popsP:
            ps = external_stream(P.stream)
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(ps)
            P.step(steps)
            b.record(ps)
            b.synchronize()
            t_sim.append(a.elapsed_time(b))
    finally:
        for P in popsP:
            P.close()
    done64 = np.cumsum(t_sim)
    cs = cells * steps
    return {"workload": f"batch{n_sims}", "simulations": n_sims, "cells": cells, "voxels": vox,
            "steps": steps, "precision": "fp32", "tuning": tuning, "autotuner": tune_info,
            "cell_steps_per_s": cs / (total_ms * 1e-3),
            "interactions_per_s": (i1 - i0) / (total_ms * 1e-3),
            "ms_per_step": total_ms / steps,
            "step_latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99))},
            "sim_completion_ms": {"p50": total_ms, "p99": total_ms},
            "phase_ms": {"binning_reorder": bin_ms, "force_update": force_ms},
            "fp64_per_simulation_path": {
                "cell_steps_per_s": cs / (sum(t_sim) * 1e-3),
                "sim_ms": {"p50": float(np.percentile(t_sim, 50)), "p99": float(np.percentile(t_sim, 99))},
                "sim_completion_ms": {"p50": float(np.percentile(done64, 50)),
                                      "p99": float(np.percentile(done64, 99))}},
            "speedup_vs_fp64_per_simulation": (cs / (total_ms * 1e-3)) / (cs / (sum(t_sim) * 1e-3)),
            "p99_completion_ratio_fp64_over_batch": float(np.percentile(done64, 99)) / total_ms}


def leg_serving(args, n_req=200, rate=50.0, budget_gib=200.0, warm=10):
    """C5: Poisson arrivals served by continuous batching from an arena sized from an HBM
    budget (FP32); the first `warm` requests are left out of the statistics."""
    import workloads
    from paper_2306_11544_amd import binding as B
    from paper_2306_11544_amd.serve import Server

    reqs = workloads.request_stream(n_req, rate)
    params = B.make_params((0, 0, 0), (1, 1, 1), c_adh=workloads.C_ADH_2, precision=B.MECH_FP32)
    pops = {r.rid: workloads.request_population(r) for r in reqs}   # drawn before the clock
    srv = Server(params, int(budget_gib * (1 << 30)), max_slots=1024, steps_per_chunk=10)
    try:
        done = srv.run(reqs, lambda r: pops[r.rid])
    finally:
        srv.close()
    measured = [d for d in done if d.rid >= warm]
    lat = np.array([d.latency_s for d in measured])
    st = srv.stats
    return {"requests": n_req, "measured_requests": len(measured), "rate_req_per_s": rate,
            "budget_gib": budget_gib, "precision": "fp32",
            "latency_s": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99))},
            "cell_steps_per_s": st["cell_steps_per_s"],
            "offered_cell_steps_per_s": sum(r.n * r.steps for r in reqs) / max(r.arrival_s for r in reqs),
            "makespan_s": st["makespan_s"], "rejected": st["rejected"],
            "max_live_slots": st["max_live_slots"], "arena_bytes": st["arena_bytes"]}


def leg_microenv(args, steps=100, cpu=True):
    """The microenvironment solver on the paper's 75^3 mesh, one oxygen-like substrate,
    FP64: the three solves of a step and the gradients."""
    import torch

    import workloads
    from paper_2306_11544_amd import binding as B

    env = workloads.microenv((75, 75, 75), 1, steps=steps)
    with B.Microenv(B.microenv_params_of(env), env.density) as M:
        M.step(5)
        M.compute_gradients()
        M.density()
        s = external_stream(M.stream)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s)
        M.step(steps)
        e1.record(s)
        e1.synchronize()
        ms_step = e0.elapsed_time(e1) / steps
        ms = M.profile(20)
    vox = env.voxels * env.n_substrates
    solve_ms = sum(ms[:3])
    bytes_step = 3 * ENV_BYTES_PER_SOLVE * vox
    gbs = bytes_step / (solve_ms * 1e-3) / 1e9
    out = {"workload": env.name, "dims": list(env.dims), "substrates": env.n_substrates,
           "ms_per_step": ms_step, "voxel_updates_per_s": vox / (ms_step * 1e-3),
           "kernel_ms": {"solve_x": ms[0], "solve_y": ms[1], "solve_z": ms[2], "gradients": ms[3]},
           "roofline": {"bound": "hbm", "kernel": "k_solve_x + k_solve_y + k_solve_z",
                        "achieved": gbs, "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": gbs / PEAK_HBM_GBS,
                        "bytes_per_voxel_step": 3 * ENV_BYTES_PER_SOLVE,
                        "gradients_GBs": ENV_BYTES_GRADIENT * vox / (ms[3] * 1e-3) / 1e9}}
    if cpu:
        from oracle import diffusion as OD
        import oracle
        p = OD.params_of(env)
        k = 5
        t0 = time.perf_counter()
        OD.step(p, env.density, k)
        t = (time.perf_counter() - t0) / k
        out["cpu_oracle"] = {"ms_per_step": t * 1e3, "voxel_updates_per_s": vox / t,
                             "cores": oracle.set_threads(0), "sample": f"{k} steps"}
    return out


def bench_batch(args):
    """The batching study alone (C4), as its own JSON line."""
    import torch
    torch.cuda.init()
    leg = leg_batch(args, n_sims=args.sims, steps=args.steps, warmup=args.warmup)
    if args.calibrate_copy_mb:
        copy_calibration(args.calibrate_copy_mb, torch.cuda.Stream(device=torch.device("cuda:0")))
    out = {"metric": "batched cell-steps/s (FP32, one launch per kernel for all simulations)",
           "value": leg["cell_steps_per_s"], "unit": "cell-steps/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": leg["ms_per_step"],
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic", "config": {"workload": leg["workload"], "simulations": leg["simulations"],
                                            "cells": leg["cells"], "precision": "fp32"}}
    out.update({k: v for k, v in leg.items() if k not in ("workload", "simulations", "cells")})
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
    ap.add_argument("--legs", default=",".join(ALL_LEGS),
                    help="extra legs of the JSON line: any of " + ",".join(ALL_LEGS) + ", or none")
    ap.add_argument("--sims", type=int, default=256, help="batch workload: simulations")
    ap.add_argument("--cells", type=int, default=0,
                    help="tumour workload with this many cells at the 1M-cell tumour's density "
                         "(core and cube scaled by (cells / 1e6)^(1/3)); a scaling study")
    ap.add_argument("--force", default="cells",
                    help="force kernel when not tuned: cells | rows | voxel | pruned")
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
    if args.workload == "microenv":
        import torch
        torch.cuda.init()
        leg = leg_microenv(args, steps=args.steps, cpu=not args.no_cpu_baseline)
        if args.calibrate_copy_mb:
            copy_calibration(args.calibrate_copy_mb, torch.cuda.Stream(device=torch.device("cuda:0")))
        print(json.dumps({"metric": "microenvironment voxel updates/s (FP64, 75^3 mesh)",
                          "value": leg["voxel_updates_per_s"], "unit": "voxel-updates/s", "n_gpus": 1,
                          "steps": args.steps, "ms_per_step": leg["ms_per_step"], "higher_is_better": True,
                          "dtype": "f64", "data": "synthetic", "config": {"workload": leg["workload"]},
                          **{k: v for k, v in leg.items() if k != "workload"}}), flush=True)
        return
    if args.locality:
        bench_locality(args)
        return
    if args.grow:
        bench_grow(args)
        return
    legs = [x for x in args.legs.split(",") if x and x != "none"]
    for x in legs:
        if x not in ALL_LEGS:
            ap.error(f"unknown leg {x}")

    import torch

    import workloads

    precision = args.precision or "fp64"
    if args.cells and args.workload == "tumour1m":
        f = (args.cells / 1e6) ** (1.0 / 3.0)
        pop = workloads.tumour(args.cells, core_radius=600.0 * f, half=1000.0 * f)
    else:
        pop = workloads.config(args.workload)
    log(f"workload {pop.name} n={pop.n} precision={precision} steps={args.steps} "
        f"warmup={args.warmup} legs={legs}")
    torch.cuda.init()
    rec, pos_main = measure_population(pop, precision, args, args.tune)
    stream = torch.cuda.Stream(device=torch.device("cuda:0"))
    if args.calibrate_copy_mb:
        copy_calibration(args.calibrate_copy_mb, stream)
    copy_gbs = copy_bandwidth(stream)
    log(f"streaming copy: {copy_gbs:.0f} GB/s")
    roof = rec["roofline"]
    roof["copy_GBs"] = copy_gbs
    roof["hbm_frac_of_copy"] = roof["hbm_algorithmic_GBs"] / copy_gbs
    roof["traffic_frac_of_copy"] = None if roof["traffic_GBs"] is None else roof["traffic_GBs"] / copy_gbs

    out = {
        "metric": METRIC,
        "value": rec["value"],
        "unit": "interactions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": rec["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32", "fp32k": "f32"}[precision],
        "data": "synthetic",
        "config": {"workload": pop.name, "cells": pop.n, "precision": precision,
                   "voxel_um": pop.voxel, "dt_min": pop.dt,
                   "integration": "f64 two-step Adams-Bashforth", "tuning": rec["tuning"],
                   "reorder_every": args.reorder_every},
        "autotuner": rec["autotuner"],
        "cell_steps_per_s": rec["cell_steps_per_s"],
        "candidates_per_s": rec["candidates_per_s"],
        "step_latency_ms": rec["step_latency_ms"],
        "phase_ms": rec["phase_ms"],
        "roofline": roof,
    }
    if "fp32k" in legs and precision != "fp32k":
        r32, pos32 = measure_population(pop, "fp32k", args, args.tune)
        d32, d64 = pos32 - pop.pos, pos_main - pop.pos
        r32["difference_from_" + precision] = {
            "steps": args.warmup + args.steps,
            "max_abs_um": float(np.abs(pos32 - pos_main).max()),
            "max_abs_over_half_width": float(np.abs(pos32 - pos_main).max() / pop.half_width),
            "displacement_relative": float(np.linalg.norm(d32 - d64) / max(np.linalg.norm(d64), 1e-300))}
        out["fp32k"] = r32
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    if "batch" in legs:
        log("leg: batch")
        out["batch"] = leg_batch(args)
        torch.cuda.empty_cache()
    if "serving" in legs:
        log("leg: serving")
        out["serving"] = leg_serving(args)
    if "microenv" in legs:
        log("leg: microenv")
        out["microenv"] = leg_microenv(args, cpu=not args.no_cpu_baseline)
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(pop, precision)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
