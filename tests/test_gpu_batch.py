"""Batches of independent simulations: each simulation's result is bitwise the same alone
(as a population) and inside a batch, whatever else runs beside it, including
simulations admitted while others are running and space reclaimed from retired ones."""
import numpy as np
import pytest

import workloads
from gpu_helpers import disp_err, pos_err, record, require_gpu, run_gpu, say
from paper_2306_11544_amd import binding as B

pytestmark = pytest.mark.gpu


def _sims(k=6, lo=800, hi=12000, seed=4000):
    sizes = workloads.batch_sizes(k, seed, lo, hi)
    return [workloads.spheroid(n, seed=seed + i, steps=0) for i, n in enumerate(sizes)]


def _params(prec, flags=0):
    # physics shared by the batch; the domain fields are not used
    return B.make_params((0, 0, 0), (1, 1, 1), c_adh=workloads.C_ADH_2, precision=prec, flags=flags)


def _capacity(pops):
    p = _params(B.MECH_FP64)
    cells = sum(pp.n for pp in pops)
    vox = sum(B.batch_request_voxels(p, pp.lo, pp.hi) for pp in pops)
    return cells, vox


@pytest.mark.parametrize("prec", [B.MECH_FP64, B.MECH_FP32_KAHAN])
def test_batch_equals_solo_bitwise(prec):
    require_gpu()
    pops = _sims()
    steps = [40, 25, 40, 10, 33, 40]
    cells, vox = _capacity(pops)
    say("batch vs solo", prec, [pp.n for pp in pops])
    with B.Batch(_params(prec), cells, vox, len(pops)) as bt:
        slots = [bt.admit_pop(pp, n_steps=s) for pp, s in zip(pops, steps)]
        bt.step(max(steps))
        B.batch_sync(bt)
        done = set(bt.poll())
        assert done == set(slots)
        got = [bt.read(s) for s in slots]
    for pp, s, (pos, vel) in zip(pops, steps, got):
        solo = run_gpu(pp, s, precision=prec)
        assert np.array_equal(pos, solo["pos"]) and np.array_equal(vel, solo["vel"])


@pytest.mark.parametrize("prec,tol", [(B.MECH_FP64, 1e-10), (B.MECH_FP32, 1e-4)])
def test_batch_matches_fp64_oracle(orc, prec, tol):
    require_gpu()
    pops = _sims(3, 1000, 5000, seed=4100)
    cells, vox = _capacity(pops)
    with B.Batch(_params(prec), cells, vox, 3) as bt:
        slots = [bt.admit_pop(pp, n_steps=60) for pp in pops]
        bt.step(60)
        got = [bt.read(s)[0] for s in slots]
    for k, (pp, g) in enumerate(zip(pops, got)):
        want = orc.run_pop(pp, steps=60)["pos"]
        err = pos_err(g, want, pp.half_width)
        record(f"batch {'fp64' if prec == B.MECH_FP64 else 'fp32'} sim{k} ({pp.n} cells) 60 steps "
               "vs fp64 oracle", err, disp_rel=disp_err(g, want, pp.pos))
        assert err <= tol


def test_batch256_full_500_steps_sampled(orc):
    """The 256-simulation batch (6.1M cells, FP32) at full size for its 500 steps: the
    smallest, the largest and four drawn simulations against the FP64 oracle."""
    require_gpu()
    pops = workloads.batch()
    cells, vox = _capacity(pops)
    say("batch256 fp32 500 steps", cells, "cells")
    with B.Batch(_params(B.MECH_FP32), cells, vox, len(pops)) as bt:
        slots = [bt.admit_pop(pp, n_steps=pp.steps) for pp in pops]
        bt.step(max(pp.steps for pp in pops))
        B.batch_sync(bt)
        assert set(bt.poll()) == set(slots)
        sizes = [pp.n for pp in pops]
        rng = np.random.default_rng(41)
        pick = sorted({int(np.argmin(sizes)), int(np.argmax(sizes)),
                       *(int(k) for k in rng.choice(len(pops), 4, replace=False))})
        got = {k: bt.read(slots[k])[0] for k in pick}
    for k in pick:
        pp = pops[k]
        say("batch256 oracle sim", k, pp.n, "cells")
        want = orc.run_pop(pp)["pos"]
        err = pos_err(got[k], want, pp.half_width)
        record(f"batch256 fp32 sim{k} ({pp.n} cells) {pp.steps} steps vs fp64 oracle", err,
               disp_rel=disp_err(got[k], want, pp.pos))
        assert err <= 1e-4, (k, err)


def test_continuous_admission_and_repack():
    """A running, B admitted while A runs, A retired, C admitted into A's space."""
    require_gpu()
    a, b, c = (workloads.spheroid(n, seed=4200 + k, steps=0)
               for k, n in enumerate((8000, 5000, 7000)))
    prec = B.MECH_FP32_KAHAN
    cap_c = a.n + b.n + 10  # C fits only once A's cells are reclaimed
    p = _params(prec)
    cap_v = max(B.batch_request_voxels(p, x.lo, x.hi) for x in (a, b, c)) * 2 + 10
    say("continuous", a.n, b.n, c.n)
    with B.Batch(p, max(cap_c, c.n + b.n), cap_v, 2) as bt:
        sa = bt.admit_pop(a, n_steps=30)
        bt.step(12)
        sb = bt.admit_pop(b, n_steps=40)   # admitted while A is mid-run
        bt.step(18)
        B.batch_sync(bt)
        assert bt.poll() == [sa]
        ra = bt.read(sa)
        with pytest.raises(B.MechError) as e:
            bt.admit_pop(c, n_steps=20)    # no free slot
        assert e.value.code == B.MECH_E_FULL
        bt.retire(sa)
        sc = bt.admit_pop(c, n_steps=20)   # reclaims A's space (compaction)
        bt.step(22)
        B.batch_sync(bt)
        assert sorted(bt.poll()) == sorted([sb, sc])
        rb = bt.read(sb)
        rc = bt.read(sc)
        info = bt.info()
        assert info["n_live"] == 2
    for pop, steps, got in ((a, 30, ra), (b, 40, rb), (c, 20, rc)):
        solo = run_gpu(pop, steps, precision=prec)
        assert np.array_equal(got[0], solo["pos"]) and np.array_equal(got[1], solo["vel"])


def test_budget_is_enforced():
    require_gpu()
    a, b = _sims(2, 2000, 4000, seed=4300)
    p = _params(B.MECH_FP32)
    va = B.batch_request_voxels(p, a.lo, a.hi)
    with B.Batch(p, a.n + 5, va + 5, 4) as bt:
        bt.admit_pop(a, n_steps=5)
        with pytest.raises(B.MechError) as e:
            bt.admit_pop(b, n_steps=5)
        assert e.value.code == B.MECH_E_BUDGET
        bt.step(5)
        B.batch_sync(bt)
        assert len(bt.poll()) == 1


@pytest.mark.parametrize("prec", [B.MECH_FP64, B.MECH_FP32])
def test_batch_graph_equals_eager(prec):
    require_gpu()
    pops = _sims(4, 1000, 6000, seed=4400)
    cells, vox = _capacity(pops)
    outs = []
    for flags in (0, B.MECH_FLAG_NO_GRAPH):
        with B.Batch(_params(prec, flags), cells, vox, 4) as bt:
            slots = [bt.admit_pop(pp, n_steps=15 + 3 * i) for i, pp in enumerate(pops)]
            for _ in range(6):
                bt.step(4)
                bt.stats()
            outs.append([bt.read(s) for s in slots])
    for (p0, v0), (p1, v1) in zip(*outs):
        assert np.array_equal(p0, p1) and np.array_equal(v0, v1)


@pytest.mark.parametrize("variant", ["rows", "voxel"])
def test_force_variants_agree(variant):
    """The kernel variants the tuner picks from agree with the default to rounding."""
    require_gpu()
    pops = _sims(3, 2000, 8000, seed=4500)
    cells, vox = _capacity(pops)
    res = {}
    for name in ("cells", variant):
        with B.Batch(_params(B.MECH_FP64, B.FORCE_KERNELS[name]), cells, vox, 3) as bt:
            slots = [bt.admit_pop(pp, n_steps=25) for pp in pops]
            bt.step(25)
            res[name] = [bt.read(s)[0] for s in slots]
    for pp, x, y in zip(pops, res["cells"], res[variant]):
        assert pos_err(x, y, pp.half_width) <= 1e-12


def test_retired_space_is_reclaimed():
    """Admitting and retiring over and over does not let retired cells pile up in the
    arena, even when it has room for them (they would still be binned every step)."""
    require_gpu()
    pops = _sims(3, 1000, 3000, seed=4650)
    p = _params(B.MECH_FP32)
    cells, vox = _capacity(pops)
    with B.Batch(p, cells * 20, vox * 20, 16) as bt:
        for _ in range(6):
            for x in pops:
                bt.admit_pop(x, n_steps=3)
            bt.step(3)
            B.batch_sync(bt)
            for s in bt.poll():
                bt.retire(s)
            info = bt.info()
            assert info["n_live"] == 0
            assert info["n_cells"] <= 2 * cells and info["n_voxels"] <= 2 * vox
