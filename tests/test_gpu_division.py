"""Growing populations on the GPU against the oracle's division rule: sizes exact, ids
and positions as the oracle's, graph and eager launches equal, cells left in place
equal to cells reordered, binning exact after growth."""
import numpy as np
import pytest

import workloads
from gpu_helpers import check_binning, pos_err, record, require_gpu, say
from paper_2306_11544_amd import binding as B

pytestmark = pytest.mark.gpu


def _grow_gpu(pop, prec, steps, cap, p_div, seed, flags=0, every=None, params=None, sizes=False):
    prm = params or B.params_of(pop, prec, flags=flags)
    with B.Population(prm, pop.pos, pop.radius, pop.type, max_cells=cap) as P:
        P.set_division(p_div, seed)
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
        binning = P.binning()
    return dict(pos=pos, vel=vel, n=n, per=per, inter=inter, binning=binning)


def _small(seed=81):
    # 1000 cells in a 200 um cube: room to grow to 1,600
    return workloads.plain(1000, seed=seed)


@pytest.mark.parametrize("prec,tol", [(B.MECH_FP64, 1e-10), (B.MECH_FP32_KAHAN, 1e-4)])
def test_growth_matches_oracle(orc, prec, tol):
    require_gpu()
    pop = _small()
    steps, cap, p_div, seed = 60, 1600, 0.008, 11
    say("grow", prec, steps)
    oprec = orc.FP64 if prec == B.MECH_FP64 else orc.FP32_KAHAN
    p = orc.params_of(pop)
    want = orc.run_growing(p, pop.pos, pop.radius, pop.type, steps=steps, precision=oprec,
                           capacity=cap, p_div=p_div, seed=seed)
    if prec == B.MECH_FP64:
        # well-posed at this horizon: a 1-ulp nudge moves the oracle far less than the bar
        nudged = orc.run_growing(p, np.nextafter(pop.pos, 0.0), pop.radius, pop.type, steps=steps,
                                 capacity=cap, p_div=p_div, seed=seed)
        assert pos_err(nudged["pos"], want["pos"], pop.half_width) <= tol / 100
    got = _grow_gpu(pop, prec, steps, cap, p_div, seed, sizes=True)
    assert got["per"] == want["per_step_n"]      # division draws depend on ids only
    assert got["n"] == want["n"] > pop.n
    err = pos_err(got["pos"], want["pos"], pop.half_width)
    record(f"grow {'fp64' if prec == B.MECH_FP64 else 'fp32k'} plain1k->{got['n']} {steps} steps", err)
    assert err <= tol, err


def test_capacity_stops_growth_by_id(orc):
    """No forces: every cell draws a division, only the five of lowest id fit."""
    require_gpu()
    pop = workloads.plain(300, seed=82)
    pos = np.clip(pop.pos, -80, 80)
    frozen = B.make_params(pop.lo, pop.hi, c_adh=[[0.0]], c_rep=0.0, precision=B.MECH_FP64)
    with B.Population(frozen, pos, pop.radius, pop.type, max_cells=pop.n + 5) as P:
        P.set_division(1.0, 5)
        P.step(1)
        assert P.size() == pop.n + 5
        got, _ = P.state()
    want = orc.run_growing(orc.params(pop.lo, pop.hi, c_rep=0.0, c_adh=((0.0,),)), pos, pop.radius,
                           steps=1, capacity=pop.n + 5, p_div=1.0, seed=5)
    np.testing.assert_allclose(got, want["pos"], rtol=0, atol=1e-12)
    np.testing.assert_allclose(np.linalg.norm(got[pop.n:] - got[:5], axis=1), pop.radius[:5],
                               rtol=1e-12)


def test_growth_graph_equals_eager():
    require_gpu()
    pop = _small(83)
    a = _grow_gpu(pop, B.MECH_FP32, 30, 1500, 0.01, 3)
    b = _grow_gpu(pop, B.MECH_FP32, 30, 1500, 0.01, 3, flags=B.MECH_FLAG_NO_GRAPH)
    assert a["n"] == b["n"]
    assert np.array_equal(a["pos"], b["pos"]) and np.array_equal(a["vel"], b["vel"])


@pytest.mark.parametrize("every", [0, 4])
def test_growth_in_place_equals_reordered(every):
    """Daughters appended at the end and left there (the paper's setting) give the same
    trajectory as reordering every step."""
    require_gpu()
    pop = workloads.spheroid(6000, seed=84, steps=0)
    a = _grow_gpu(pop, B.MECH_FP32_KAHAN, 40, 9000, 0.01, 21)
    b = _grow_gpu(pop, B.MECH_FP32_KAHAN, 40, 9000, 0.01, 21, every=every)
    assert a["n"] == b["n"] > pop.n
    assert np.array_equal(a["pos"], b["pos"]) and np.array_equal(a["vel"], b["vel"])
    assert a["inter"] == b["inter"]


def test_binning_after_growth_is_exact(orc):
    require_gpu()
    pop = _small(85)
    prm = B.params_of(pop, B.MECH_FP64)
    with B.Population(prm, pop.pos, pop.radius, pop.type, max_cells=1500) as P:
        P.set_division(0.02, 8)
        P.step(10)
        before, _ = P.state()
        P.set_division(0.0)
        P.step(1)
        vid, start, ids, occ = P.binning()
    want = orc.bin(orc.params_of(pop), before)
    check_binning((vid, start, ids, occ), want, before, pop.lo, pop.hi, pop.voxel)


def test_bad_division_arguments():
    require_gpu()
    pop = workloads.plain()
    with B.Population(B.params_of(pop, B.MECH_FP64), pop.pos, pop.radius, pop.type) as P:
        for bad in (-0.1, 1.5, float("nan")):
            with pytest.raises(B.MechError) as e:
                P.set_division(bad, 1)
            assert e.value.code == B.MECH_E_INVALID
        # without room to grow, division is accepted and simply adds no cells
        P.set_division(0.5, 1)
        P.step(3)
        assert P.size() == pop.n
    with pytest.raises(B.MechError):
        B.Population(B.params_of(pop, B.MECH_FP64), pop.pos, pop.radius, pop.type,
                     max_cells=pop.n - 1)
