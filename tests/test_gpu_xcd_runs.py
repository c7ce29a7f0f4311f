"""Runs of equal measured work: on grids that fill every resident slot, each XCD takes a
run of the sorted cells cut from the last launch's wave durations.  The cut moves which
workgroup takes a cell, never a result: a population stepped with it equals, bitwise,
the same population on a grid too small to use it, and the cut lies ordered inside the
population."""
import numpy as np
import pytest

import workloads
from gpu_helpers import require_gpu, say
from paper_2306_11544_amd import binding as B

pytestmark = pytest.mark.gpu

N = 600_000   # 9375 one-wave tiles: more than the 8192 resident slots of the chip


def _tumour():
    s = (N / 1e6) ** (1.0 / 3.0)   # the 1M-cell tumour's density
    return workloads.tumour(N, seed=77, steps=0, core_radius=600.0 * s, half=1000.0 * s)


def _run(pop, prec, tuning, steps):
    with B.Population(B.params_of(pop, prec), pop.pos, pop.radius, pop.type) as P:
        P.set_tuning(tuning)
        P.step(steps)
        pos, vel = P.state()
        split = P.xcd_split()
        _, inter, cand = P.stats()
    return pos, vel, split, inter, cand


@pytest.mark.parametrize("prec", [B.MECH_FP64, B.MECH_FP32_KAHAN])
def test_cut_runs_equal_uncut_bitwise(prec):
    require_gpu()
    pop = _tumour()
    say("xcd runs", N, "cells, precision", prec)
    cut = _run(pop, prec, B.tuning(0, 1, 8, 0, 0), 6)
    # one workgroup per compute unit: too few to cut, the equal-count runs
    flat = _run(pop, prec, B.tuning(0, 1, 8, 1, 0), 6)
    split = cut[2]
    # the tumour's end runs hold its sparse outer cells: the cut is kept
    assert split[8] == N, split
    assert split[0] == 0 and np.all(np.diff(split[:8].astype(np.int64)) >= 0) and split[7] <= N, split
    assert flat[2][8] == 0, flat[2]
    assert np.array_equal(cut[0], flat[0])
    assert np.array_equal(cut[1], flat[1])
    assert cut[3:] == flat[3:]
