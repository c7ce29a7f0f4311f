"""Shared helpers of the GPU parity tests (not collected: no test_ prefix)."""
import sys

import numpy as np

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


def pos_err(a, b, S):
    """Domain-scaled position error: max over cells and axes of |a - b| / S."""
    if a.size == 0:
        return 0.0
    return float(np.abs(a - b).max() / S)
