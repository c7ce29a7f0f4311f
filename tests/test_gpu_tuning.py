"""Force-kernel launch configurations (what the autotuner picks from): every one gives
the default's results up to summation order, each is deterministic, bad values are
rejected, and the tuner's choice is cached per shape class."""
import json

import numpy as np
import pytest

import workloads
from gpu_helpers import pos_err, require_gpu, say
from paper_2306_11544_amd import autotune as A
from paper_2306_11544_amd import binding as B

pytestmark = pytest.mark.gpu


def _sims(k=3, lo=2000, hi=6000, seed=4600):
    sizes = workloads.batch_sizes(k, seed, lo, hi)
    return [workloads.spheroid(n, seed=seed + i, steps=0) for i, n in enumerate(sizes)]


def _params(prec=B.MECH_FP64):
    return B.make_params((0, 0, 0), (1, 1, 1), c_adh=workloads.C_ADH_2, precision=prec)


def _run(pops, t, steps, prec=B.MECH_FP64):
    p = _params(prec)
    cells = sum(x.n for x in pops)
    vox = sum(B.batch_request_voxels(p, x.lo, x.hi) for x in pops)
    with B.Batch(p, cells, vox, len(pops)) as bt:
        bt.set_tuning(t)
        got = bt.get_tuning().as_dict()
        assert got == t.as_dict()
        slots = [bt.admit_pop(x, n_steps=steps) for x in pops]
        bt.step(1)
        _, inter1, _ = bt.stats()
        bt.step(steps - 1)
        res = [bt.read(s) for s in slots]
    return res, inter1


def test_every_configuration_agrees_with_default():
    require_gpu()
    pops = _sims()
    ref, inter_ref = _run(pops, A.DEFAULT, 12)
    for t in A.search_space():
        say("tuning", t.as_dict())
        got, inter = _run(pops, t, 12)
        assert inter == inter_ref  # first-step decisions do not depend on the order
        for pp, (p0, _), (p1, _) in zip(pops, ref, got):
            assert pos_err(p1, p0, pp.half_width) <= 1e-12


@pytest.mark.parametrize("prec", [B.MECH_FP64, B.MECH_FP32, B.MECH_FP32_KAHAN])
def test_list_kernel_equals_inline_kernel_bitwise(prec):
    """The list kernel's prefilter and slab window (or, pruned, its row test and trimmed
    windows) drop no interacting pair and its lists keep the neighbour order: at every
    list length and tile its trajectories are bitwise those of the inline kernel, which
    evaluates every pair of the 27 voxels in order."""
    require_gpu()
    pops = _sims(3, 3000, 8000, seed=4650)
    ref, inter_ref = _run(pops, B.tuning("rows", 4, 4, 0), 15, prec)
    for cfg in [("cells", 4, 4, 0, 16), ("cells", 4, 4, 0, 32), ("cells", 4, 4, 0, 64),
                ("cells", 1, 8, 0, 64), ("cells", 8, 2, 16, 32), ("cells", 2, 8, 0, 16),
                ("pruned", 4, 4, 0, 16), ("pruned", 1, 8, 0, 32), ("pruned", 2, 2, 0, 64)]:
        say("list kernel", prec, cfg)
        got, inter = _run(pops, B.tuning(*cfg), 15, prec)
        assert inter == inter_ref
        for (p0, v0), (p1, v1) in zip(ref, got):
            assert np.array_equal(p0, p1) and np.array_equal(v0, v1), cfg


@pytest.mark.parametrize("cfg", [("cells", 8, 2, 16), ("cells", 1, 8, 0), ("rows", 2, 4, 0),
                                 ("voxel", 4, 4, 2)])
def test_configuration_is_deterministic(cfg):
    require_gpu()
    pops = _sims(2, 3000, 5000, seed=4700)
    t = B.tuning(*cfg)
    a, _ = _run(pops, t, 8, B.MECH_FP32_KAHAN)
    b, _ = _run(pops, t, 8, B.MECH_FP32_KAHAN)
    for (p0, v0), (p1, v1) in zip(a, b):
        assert np.array_equal(p0, p1) and np.array_equal(v0, v1)


def test_bad_configurations_are_rejected():
    require_gpu()
    pops = _sims(1, 1000, 1000, seed=4800)
    p = _params()
    with B.Batch(p, pops[0].n, B.batch_request_voxels(p, pops[0].lo, pops[0].hi), 1) as bt:
        for bad in (B.tuning(6, 4, 4, 0), B.tuning(10, 4, 4, 0), B.tuning(0, 3, 4, 0), B.tuning(0, 16, 4, 0),
                    B.tuning(0, 4, 16, 0), B.tuning(0, 4, 1, 0), B.tuning(0, 4, 4, 65),
                    B.tuning(0, 4, 4, -1), B.tuning(0, 4, 4, 0, 20), B.tuning(0, 4, 4, 0, 48),
                    B.tuning(0, 8, 4, 0, 64)):
            with pytest.raises(B.MechError) as e:
                bt.set_tuning(bad)
            assert e.value.code == B.MECH_E_INVALID
        assert bt.get_tuning().as_dict() == A.DEFAULT.as_dict()


def test_tuner_choice_is_cached(tmp_path, monkeypatch):
    require_gpu()
    monkeypatch.setenv("MECH_TUNE_CACHE", str(tmp_path / "tuning.json"))
    pops = _sims(2, 2000, 4000, seed=4900)
    p = _params(B.MECH_FP32)
    space = [B.tuning("cells", 4, 4, 0), B.tuning("cells", 2, 8, 0), B.tuning("rows", 4, 4, 0)]
    best = A.tuned(p, pops, space=space, steps=2, repeats=1)
    assert best.as_dict() in [t.as_dict() for t in space]
    data = json.load(open(tmp_path / "tuning.json"))
    key = A.shape_class(p, pops)
    assert data[key]["tuning"] == best.as_dict()
    # a second call is answered from the cache (an empty space would fail if it tuned)
    again = A.tuned(p, pops, space=[object()])
    assert again.as_dict() == best.as_dict()


def test_population_tuning():
    require_gpu()
    pop = workloads.plain()
    prm = B.params_of(pop, B.MECH_FP64)
    outs = []
    for t in (A.DEFAULT, B.tuning("cells", 2, 2, 8), B.tuning("voxel", 4, 4, 4)):
        with B.Population(prm, pop.pos, pop.radius, pop.type) as P:
            P.set_tuning(t)
            assert P.get_tuning().as_dict() == t.as_dict()
            P.step(20)
            outs.append(P.state()[0])
    for o in outs[1:]:
        assert pos_err(o, outs[0], pop.half_width) <= 1e-12


@pytest.mark.parametrize("case", ["core", "pile", "sparse"])
def test_staged_rows_equal_inline_kernel_bitwise(case):
    """The one-type FP64 list kernel stages a wave's shared rows in LDS: in a dense core
    (rows staged), a pile denser than the stage holds (rows walked from memory in the
    same waves) and scattered cells (waves spanning two rows), its trajectories are
    bitwise those of the inline kernel, at several shapes."""
    require_gpu()
    if case == "core":
        s = 0.2 ** (1.0 / 3.0)   # the 1M-cell tumour's density at 200k cells
        pop = workloads.tumour(200_000, seed=81, steps=0, core_radius=600.0 * s, half=1000.0 * s)
    elif case == "pile":
        pop = workloads.plain(12_000, seed=82, steps=0, half=45.0)   # ~440 cells per voxel
    else:
        pop = workloads.plain(20_000, seed=83, steps=0, half=600.0)
    p = B.params_of(pop, B.MECH_FP64)

    def run(t):
        with B.Population(p, pop.pos, pop.radius, pop.type) as P:
            P.set_tuning(t)
            P.step(6)
            pos, vel = P.state()
            _, inter, _ = P.stats()
        return pos, vel, inter

    say("staged rows", case, pop.n)
    ref = run(B.tuning("rows", 4, 4, 0))
    for cfg in [("cells", 1, 8, 0, 16), ("cells", 4, 4, 0, 16), ("cells", 2, 8, 0, 32), ("cells", 1, 2, 0, 64)]:
        got = run(B.tuning(*cfg))
        assert got[2] == ref[2], cfg
        assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1]), cfg
