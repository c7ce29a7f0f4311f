"""Shared helpers of the GPU parity tests (not collected: no test_ prefix)."""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

from paper_2306_11544_amd import binding as B


def say(*a):
    """Name the case before a GPU step, flushed, so a crash log points at it."""
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


def require_gpu():
    n = B.mech_device_count()
    assert n > 0, "no HIP device visible to libmech.so"


def run_gpu(pop, steps, precision=B.MECH_FP64, ab2_start=B.MECH_AB2_ZERO_HISTORY, flags=0,
            per_step=False, prev_velocity=None):
    """Run `steps` steps; returns dict(pos, vel, interactions, candidates[, per_step])."""
    p = B.params_of(pop, precision, ab2_start, flags)
    with B.Population(p, pop.pos, pop.radius, pop.type, prev_velocity) as P:
        per = []
        if per_step:
            last = 0
            for _ in range(steps):
                P.step(1)
                _, it, _ = P.stats()
                per.append(it - last)
                last = it
        else:
            P.step(steps)
        pos, vel = P.state()
        s, it, cand = P.stats()
        assert s == steps
    out = dict(pos=pos, vel=vel, interactions=it, candidates=cand)
    if per_step:
        out["per_step"] = np.array(per, dtype=np.int64)
    return out


def record(case, err, **extra):
    """Append a parity error to the JSON-lines file named by MECH_PARITY_LOG, if set:
    the per-configuration error table is collected this way."""
    out = os.environ.get("MECH_PARITY_LOG")
    if out and os.path.isdir(os.path.dirname(os.path.abspath(out))):
        with open(out, "a") as f:
            f.write(json.dumps({"case": case, "err": float(err), **extra}) + "\n")


def assert_well_posed(orc, pop, steps, bar=1e-10):
    """The oracle's own trajectory moves by far less than the bar when every input
    coordinate is nudged by one ulp, and when the cells are relabelled (which changes
    the order of every force sum).  Otherwise the case is chaotic at this horizon and
    no implementation that sums in another order could be held to the bar."""
    p = orc.params_of(pop)
    a = orc.run(p, pop.pos, pop.radius, pop.type, steps=steps)["pos"]
    b = orc.run(p, np.nextafter(pop.pos, 0.0), pop.radius, pop.type, steps=steps)["pos"]
    perm = np.random.default_rng(0).permutation(pop.n)
    c = np.empty_like(a)
    c[perm] = orc.run(p, pop.pos[perm], pop.radius[perm], pop.type[perm], steps=steps)["pos"]
    sens = max(pos_err(a, b, pop.half_width), pos_err(a, c, pop.half_width))
    assert sens <= bar / 100, f"ill-posed case: sensitivity {sens:.2e}"


def pos_err(a, b, S):
    """Domain-scaled position error: max over cells and axes of |a - b| / S."""
    if a.size == 0:
        return 0.0
    return float(np.abs(a - b).max() / S)
