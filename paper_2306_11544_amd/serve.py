"""Continuous-batching server for simulation requests on one GPU.

Requests (a population and a step count each) arrive over time.  The server keeps one
batch (see include/mech.h) whose arena is sized from an HBM budget: a request is
admitted as soon as it has arrived and its cells and voxels fit in the space the
running simulations leave free (first come, first served), and, if a live-cell limit is
set, while the cells already running stay below it; it then runs inside the same
step launches as every other admitted request, its state stays on the device, and it
is read back and retired when its last step completes.  Requests that do not fit wait
in the queue until earlier ones finish.  Each request's result is bitwise the one it
would get alone.

The loop enqueues a chunk of steps, admits arrivals while that chunk runs (admission
copies go on a second stream), waits for the chunk and reads the finished requests.
Each request stops at its own step count inside a chunk (its slot freezes on the
device), so chunks keep a fixed length whatever the requests still need.
Latency is completion minus arrival.  Completion is the device time of the request's
last step (its slot's completion event, measured against a clock mark taken when the
loop starts), not the end of the chunk it finished in, so a request that ends early in
a chunk is not charged the rest of it.  A request larger than the whole arena can never
be admitted: it is rejected (recorded in `rejected`) instead of waiting forever.

  python -m paper_2306_11544_amd.serve --requests 400 --rate 50 --budget-gb 200
"""
from __future__ import annotations

import argparse
import collections
import json
import sys
import time
from dataclasses import dataclass, field

import numpy as np

from . import binding as B


@dataclass
class Done:
    rid: int
    n: int
    steps: int
    arrival_s: float
    admit_s: float
    done_s: float
    pos: np.ndarray | None = None
    vel: np.ndarray | None = None

    @property
    def latency_s(self) -> float:
        return self.done_s - self.arrival_s


def capacity_for_budget(params: B.MechParams, budget_bytes: int, voxels_per_cell: float,
                        max_slots: int):
    """Largest (cells, voxels) arena, voxels = voxels_per_cell * cells, within the budget
    (the library's batch_budget_capacity)."""
    return B.batch_budget_capacity(params, budget_bytes, voxels_per_cell, max_slots)


@dataclass
class Server:
    params: B.MechParams
    budget_bytes: int
    max_slots: int = 1024
    voxels_per_cell: float = 1.6
    steps_per_chunk: int = 10
    # Cells allowed on the device at once (None: as many as the budget holds).  Every
    # live request advances one step per batch step, so the more run together, the
    # slower each one goes; once the GPU is saturated (a few million cells), admitting
    # more adds latency and no throughput.
    max_live_cells: int | None = None
    stats: dict = field(default_factory=dict)

    def __post_init__(self):
        self.batch = self.make_batch()
        cap = self.batch.capacity()
        self.cap_cells, self.cap_voxels = cap["max_cells"], cap["max_voxels"]
        self.arena_bytes = cap["arena_bytes"]
        self.rejected = []

    def make_batch(self):
        """The batch whose arena the library sizes from the HBM budget."""
        return B.Batch(self.params, max_slots=self.max_slots, budget_bytes=self.budget_bytes,
                       voxels_per_cell=self.voxels_per_cell)

    def close(self):
        self.batch.close()

    def run(self, requests, make_population, keep_results=False, log=None):
        """Serve `requests` (objects with rid, arrival_s, n, steps) in real time.

        make_population(request) builds its workloads.Population.  Returns the list of
        Done records in completion order."""
        bt = self.batch
        pending = collections.deque(sorted(requests, key=lambda r: r.arrival_s))
        queue = collections.deque()
        running = {}   # slot -> (request, population size, admit time)
        done = []
        cell_steps = 0
        live_cells = 0
        max_live = 0
        max_queue = 0
        busy_chunks = 0
        bt.mark_clock()
        t0 = time.perf_counter()   # the device reached the clock mark just before this

        def now():
            return time.perf_counter() - t0

        while pending or queue or running:
            t = now()
            while pending and pending[0].arrival_s <= t:
                r = pending.popleft()
                queue.append((r, make_population(r)))
            max_queue = max(max_queue, len(queue))
            # enqueue a chunk of steps for the admitted requests; a request whose steps
            # run out inside the chunk freezes on the device at its own last step
            if running:
                bt.step(self.steps_per_chunk)
                busy_chunks += 1
            # admit while the chunk runs: first come, first served
            while queue:
                r, pop = queue[0]
                if (self.max_live_cells is not None and running
                        and live_cells + pop.n > self.max_live_cells):
                    break
                try:
                    slot = bt.admit_pop(pop, n_steps=r.steps)
                except B.MechError as e:
                    if e.code not in (B.MECH_E_BUDGET, B.MECH_E_FULL):
                        raise
                    if running:
                        break           # waits for running requests to free space
                    # nothing runs and it still does not fit: it never will
                    queue.popleft()
                    self.rejected.append((r.rid, pop.n, str(e)))
                    if log:
                        log(f"rejected rid={r.rid} n={pop.n}: {e}")
                    continue
                queue.popleft()
                running[slot] = (r, pop.n, now())
                live_cells += pop.n
            max_live = max(max_live, len(running))
            bt.sync()
            for slot in bt.poll():
                r, n, t_admit = running.pop(slot)
                live_cells -= n
                t_done = bt.done_ms(slot) * 1e-3
                pos = vel = None
                if keep_results:
                    pos, vel = bt.read(slot)
                bt.retire(slot)
                cell_steps += n * r.steps
                done.append(Done(r.rid, n, r.steps, r.arrival_s, t_admit, t_done, pos, vel))
                if log:
                    log(f"done rid={r.rid} n={n} steps={r.steps} latency={t_done - r.arrival_s:.3f}s")
            if not running and not queue and pending:
                time.sleep(max(0.0, min(0.01, pending[0].arrival_s - now())))
        makespan = now()
        lat = np.array([d.latency_s for d in done]) if done else np.zeros(1)
        self.stats = {
            "requests": len(done),
            "rejected": len(self.rejected),
            "makespan_s": makespan,
            "cell_steps": cell_steps,
            "cell_steps_per_s": cell_steps / makespan if makespan > 0 else 0.0,
            "latency_p50_s": float(np.percentile(lat, 50)),
            "latency_p99_s": float(np.percentile(lat, 99)),
            "latency_mean_s": float(lat.mean()),
            "max_live_slots": max_live,
            "max_queue": max_queue,
            "chunks": busy_chunks,
            "max_live_cells": self.max_live_cells,
            "arena_bytes": self.arena_bytes,
            "cap_cells": self.cap_cells,
            "cap_voxels": self.cap_voxels,
        }
        return done


def main(argv=None):
    import os
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import workloads

    ap = argparse.ArgumentParser()
    ap.add_argument("--requests", type=int, default=400)
    ap.add_argument("--warmup", type=int, default=20, help="requests excluded from the statistics")
    ap.add_argument("--rate", type=float, default=50.0)
    ap.add_argument("--budget-gb", type=float, default=200.0, help="HBM budget in GiB")
    ap.add_argument("--precision", default="fp32")
    ap.add_argument("--chunk", type=int, default=10)
    ap.add_argument("--max-slots", type=int, default=1024)
    ap.add_argument("--max-live-cells", type=int, default=0,
                    help="cells on the device at once (0: as many as the budget holds)")
    args = ap.parse_args(argv)
    reqs = workloads.request_stream(args.requests, args.rate)
    params = B.make_params((0, 0, 0), (1, 1, 1), c_adh=workloads.C_ADH_2,
                           precision=B.PRECISIONS[args.precision])
    srv = Server(params, int(args.budget_gb * (1 << 30)), args.max_slots,
                 steps_per_chunk=args.chunk, max_live_cells=args.max_live_cells or None)
    # populations are drawn before the clock starts
    pops = {r.rid: workloads.request_population(r) for r in reqs}
    done = srv.run(reqs, lambda r: pops[r.rid])
    srv.close()
    measured = [d for d in done if d.rid >= args.warmup]
    lat = np.array([d.latency_s for d in measured])
    offered = sum(r.n * r.steps for r in reqs) / max(r.arrival_s for r in reqs)
    out = dict(srv.stats)
    out.update({
        "measured_requests": len(measured),
        "latency_p50_s": float(np.percentile(lat, 50)),
        "latency_p99_s": float(np.percentile(lat, 99)),
        "offered_cell_steps_per_s": offered,
        "rate_req_per_s": args.rate,
        "budget_gib": args.budget_gb,
        "precision": args.precision,
    })
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
