"""One-type FP64 arenas keep a record (x, y, z, r) per cell, which the one-type force
kernels' evaluation reads in place of four gathers; the inline kernel (every pair of the
27 voxels) reads the four arrays.  Results must be the same bit for bit whichever writes
the records: the gather of a large population is covered by the staged-rows tests, and
here
* the gather of a batch of one-type simulations (records at each slot's cells),
  against each simulation run alone;
* the one-workgroup binning of a small population, against the inline kernel;
* the shadow kernel of cells left in place (records in storage order, candidates read
  through the sorted index), against the same population reordered every step."""
import numpy as np
import pytest

import workloads
from gpu_helpers import require_gpu, run_gpu, say
from paper_2306_11544_amd import binding as B

pytestmark = pytest.mark.gpu


def _run(pop, steps, tuning=None, every=None):
    with B.Population(B.params_of(pop, B.MECH_FP64), pop.pos, pop.radius, pop.type) as P:
        if tuning is not None:
            P.set_tuning(tuning)
        if every is not None:
            P.set_reorder(every)
        P.step(steps)
        pos, vel = P.state()
        _, inter, cand = P.stats()
    return pos, vel, inter


def test_records_of_small_population_equal_inline_kernel_bitwise():
    require_gpu()
    pop = workloads.plain(5_000, seed=91, steps=0, half=150.0)   # one workgroup bins it
    assert pop.n_types == 1
    say("fp64 records, small population", pop.n)
    ref = _run(pop, 20, B.tuning("rows", 4, 4, 0))
    got = _run(pop, 20, B.tuning("cells", 1, 8, 0, 16))
    assert ref[2] > 0 and got[2] == ref[2]
    assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1])


def test_records_of_cells_left_in_place_bitwise():
    require_gpu()
    s = 0.6 ** (1.0 / 3.0)   # the 1M-cell tumour's density at 600k cells
    pop = workloads.tumour(600_000, seed=93, steps=0, core_radius=600.0 * s, half=1000.0 * s)
    say("fp64 records in place", pop.n)
    ref = _run(pop, 6)
    got = _run(pop, 6, every=0)
    assert ref[2] > 0 and got[2] == ref[2]
    assert np.array_equal(ref[0], got[0]) and np.array_equal(ref[1], got[1])


def test_records_in_a_one_type_batch_equal_solo_bitwise():
    require_gpu()
    s = 0.01 ** (1.0 / 3.0)   # the 1M-cell tumour's density at 10k cells
    pops = [workloads.tumour(n, seed=94 + k, steps=0, core_radius=600.0 * s, half=1000.0 * s)
            for k, n in enumerate((10_000, 4_000, 7_000))]
    steps = [25, 12, 25]
    p = B.make_params((0, 0, 0), (1, 1, 1), c_adh=workloads.C_ADH_1, precision=B.MECH_FP64)
    cells = sum(pp.n for pp in pops)
    vox = sum(B.batch_request_voxels(p, pp.lo, pp.hi) for pp in pops)
    say("fp64 records, one-type batch", [pp.n for pp in pops])
    with B.Batch(p, cells, vox, len(pops)) as bt:
        slots = [bt.admit_pop(pp, n_steps=k) for pp, k in zip(pops, steps)]
        bt.step(max(steps))
        B.batch_sync(bt)
        assert set(bt.poll()) == set(slots)
        got = [bt.read(sl) for sl in slots]
    for pp, k, (pos, vel) in zip(pops, steps, got):
        solo = run_gpu(pp, k, precision=B.MECH_FP64)
        assert np.array_equal(pos, solo["pos"]) and np.array_equal(vel, solo["vel"])
