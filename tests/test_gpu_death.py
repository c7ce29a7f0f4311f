"""Populations that divide and die on the GPU against the oracle's rules: sizes exact
step by step, positions as the oracle's, graph and eager launches equal, cells left in
place equal to cells reordered, binning exact after deaths, a population that dies out."""
import numpy as np
import pytest

import workloads
from gpu_helpers import check_binning, pos_err, record, require_gpu, say
from paper_2306_11544_amd import binding as B

pytestmark = pytest.mark.gpu


def _turnover_gpu(pop, prec, steps, cap, p_div, p_death, seed, flags=0, every=None, sizes=False):
    prm = B.params_of(pop, prec, flags=flags)
    with B.Population(prm, pop.pos, pop.radius, pop.type, max_cells=cap) as P:
        P.set_division(p_div, seed)
        P.set_death(p_death)
        if every is not None:
            P.set_reorder(every)
        per = []
        if sizes:
            for _ in range(steps):
                P.step(1)
                per.append(P.size())
        else:
            P.step(steps)
        pos, vel = P.state()
        n = P.size()
        _, inter, _ = P.stats()
    return dict(pos=pos, vel=vel, n=n, per=per, inter=inter)


@pytest.mark.parametrize("prec,tol", [(B.MECH_FP64, 1e-10), (B.MECH_FP32_KAHAN, 1e-4)])
def test_turnover_matches_oracle(orc, prec, tol):
    require_gpu()
    pop = workloads.plain(1000, seed=91)
    steps, cap, p_div, p_death, seed = 60, 1600, 0.01, 0.006, 17
    say("turnover", prec, steps)
    oprec = orc.FP64 if prec == B.MECH_FP64 else orc.FP32_KAHAN
    want = orc.run_growing(orc.params_of(pop), pop.pos, pop.radius, pop.type, steps=steps,
                           precision=oprec, capacity=cap, p_div=p_div, seed=seed, p_death=p_death)
    got = _turnover_gpu(pop, prec, steps, cap, p_div, p_death, seed, sizes=True)
    assert got["per"] == want["per_step_n"]      # both draws depend on ids only
    # the population both shrank and grew on the way
    assert min(np.diff([pop.n] + got["per"])) < 0 < max(np.diff([pop.n] + got["per"]))
    err = pos_err(got["pos"], want["pos"], pop.half_width)
    record(f"turnover {'fp64' if prec == B.MECH_FP64 else 'fp32k'} plain1k->{got['n']} {steps} steps", err)
    assert err <= tol, err


def test_death_only_matches_oracle(orc):
    """Death without division, 2 types: survivors keep id order, radius and type."""
    require_gpu()
    pop = workloads.tumour(3000, seed=92)
    steps, p_death, seed = 25, 0.02, 4
    want = orc.run_growing(orc.params_of(pop), pop.pos, pop.radius, pop.type, steps=steps,
                           p_death=p_death, seed=seed)
    prm = B.params_of(pop, B.MECH_FP64)
    with B.Population(prm, pop.pos, pop.radius, pop.type) as P:
        P.set_division(0.0, seed)
        P.set_death(p_death)
        P.step(steps)
        n = P.size()
        pos, _ = P.state()
    assert n == want["n"] < pop.n
    assert pos_err(pos, want["pos"], pop.half_width) <= 1e-10


def test_turnover_graph_equals_eager():
    require_gpu()
    pop = workloads.plain(1000, seed=93)
    a = _turnover_gpu(pop, B.MECH_FP32, 30, 1500, 0.01, 0.01, 3)
    b = _turnover_gpu(pop, B.MECH_FP32, 30, 1500, 0.01, 0.01, 3, flags=B.MECH_FLAG_NO_GRAPH)
    assert a["n"] == b["n"]
    assert np.array_equal(a["pos"], b["pos"]) and np.array_equal(a["vel"], b["vel"])


@pytest.mark.parametrize("every", [0, 4])
def test_turnover_in_place_equals_reordered(every):
    require_gpu()
    pop = workloads.spheroid(6000, seed=94, steps=0)
    a = _turnover_gpu(pop, B.MECH_FP32_KAHAN, 40, 9000, 0.01, 0.008, 21)
    b = _turnover_gpu(pop, B.MECH_FP32_KAHAN, 40, 9000, 0.01, 0.008, 21, every=every)
    assert a["n"] == b["n"]
    assert np.array_equal(a["pos"], b["pos"]) and np.array_equal(a["vel"], b["vel"])
    assert a["inter"] == b["inter"]


def test_binning_after_deaths_is_exact(orc):
    require_gpu()
    pop = workloads.plain(1000, seed=95)
    prm = B.params_of(pop, B.MECH_FP64)
    with B.Population(prm, pop.pos, pop.radius, pop.type, max_cells=1500) as P:
        P.set_division(0.01, 8)
        P.set_death(0.03)
        P.step(10)
        before, _ = P.state()
        assert len(before) < pop.n
        P.set_division(0.0, 8)
        P.set_death(0.0)
        P.step(1)
        vid, start, ids, occ = P.binning()
    want = orc.bin(orc.params_of(pop), before)
    check_binning((vid, start, ids, occ), want, before, pop.lo, pop.hi, pop.voxel)


def test_population_dies_out():
    """p_death = 1: every cell dies in the first step; later steps run on no cells, and
    the step count keeps going."""
    require_gpu()
    pop = workloads.plain(500, seed=96)
    with B.Population(B.params_of(pop, B.MECH_FP32), pop.pos, pop.radius, pop.type) as P:
        P.set_death(1.0)
        P.step(1)
        assert P.size() == 0
        P.step(5)
        assert P.size() == 0
        pos, vel = P.state()
        assert pos.shape == (0, 3) and vel.shape == (0, 3)
        steps, inter, _ = P.stats()
        assert steps == 6


def test_bad_death_arguments():
    require_gpu()
    pop = workloads.plain(300, seed=97)
    with B.Population(B.params_of(pop, B.MECH_FP64), pop.pos, pop.radius, pop.type) as P:
        for bad in (-0.1, 1.5, float("nan")):
            with pytest.raises(B.MechError) as e:
                P.set_death(bad)
            assert e.value.code == B.MECH_E_INVALID
