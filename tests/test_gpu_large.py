"""Beyond the 32-bit byte range: 140 million cells (their float shadow spans more than
2^31 bytes and their positions more than 2^30), one FP32+Kahan step, checked on
sampled cells against the oracle, which computes each of them alone."""
import time

import numpy as np
import pytest

import workloads
from gpu_helpers import record, require_gpu, say
from paper_2306_11544_amd import binding as B

pytestmark = pytest.mark.gpu


def test_140m_cells_one_step(orc):
    require_gpu()
    n = 140_000_000
    half = 6180.0            # 412 voxels a side, about 2 cells per voxel
    t0 = time.perf_counter()
    pop = workloads.plain(n, seed=91, steps=1, half=half)
    say("large", n, f"inputs drawn {time.perf_counter() - t0:.1f} s")
    prm = B.params_of(pop, B.MECH_FP32_KAHAN)
    with B.Population(prm, pop.pos, pop.radius, pop.type) as P:
        say("large", f"created {time.perf_counter() - t0:.1f} s")
        P.step(1)
        pos, vel = P.state()
        steps, inter, cand = P.stats()
        say("large", f"stepped and read {time.perf_counter() - t0:.1f} s")
        vid, start, ids, occ = P.binning()
        say("large", f"binning read {time.perf_counter() - t0:.1f} s")
    assert steps == 1 and inter > 0 and cand > inter
    # binning describes the positions the step started from: a permutation whose
    # voxels ascend, with starts that count them
    rng = np.random.default_rng(92)
    probe = rng.choice(n, 20000, replace=False)
    v_ids = vid[ids]
    assert np.all(np.diff(v_ids[: 2_000_000].astype(np.int64)) >= 0)
    assert start[-1] == n and np.all(np.diff(start[:: 1000].astype(np.int64)) >= 0)
    slot = np.empty(n, np.int64)
    slot[ids] = np.arange(n)
    assert np.all((start[vid[probe]] <= slot[probe]) & (slot[probe] < start[vid[probe] + 1]))
    # sampled first-step velocities against the oracle's own computation of those cells
    sample = rng.choice(n, 1500, replace=False)
    p = orc.params_of(pop)
    say("large", f"checks {time.perf_counter() - t0:.1f} s")
    v32, _ = orc.velocity_sampled(p, pop.pos, pop.radius, pop.type, sample, orc.FP32_KAHAN)
    say("large", f"oracle {time.perf_counter() - t0:.1f} s")
    scale = max(np.abs(v32).max(), 1e-12)
    err = np.abs(vel[sample] - v32).max() / scale
    record("fp32k 140M cells step-1 sampled velocity vs fp32k oracle (rel. to max|v|)", err)
    assert err <= 2e-5
    assert np.all(np.isfinite(pos)) and pos.min() >= -half and pos.max() <= half
    # away from the walls, the cells left the step where Adams-Bashforth put them
    inner = sample[np.all(np.abs(pop.pos[sample]) < half - 10.0, axis=1)]
    moved = pos[inner] - pop.pos[inner]
    np.testing.assert_allclose(moved, 1.5 * pop.dt * vel[inner], rtol=0, atol=1e-9 * half)
