"""The allocation-free entry point (step_mechanics_noalloc) against the population path
(create_population + step_mechanics + read_state) through the C ABI: the same kernels in
the same order, so the results must be bitwise equal.  Two calls in a row, the second
with a smaller input, so the second runs on the scratch the first left behind."""
import numpy as np
import pytest

import workloads
from gpu_helpers import require_gpu, say
from paper_2306_11544_amd import binding as B

pytestmark = pytest.mark.gpu


def _population_path(prm, pop, steps, vprev=None):
    with B.Population(prm, pop.pos, pop.radius, pop.type, vprev) as P:
        P.step(steps)
        pos, vel = P.state()
        _, inter, _ = P.stats()
    return pos, vel, inter


def _subset(pop, n, name):
    return workloads.Population(name, pop.pos[:n].copy(), pop.radius[:n].copy(), pop.type[:n].copy(),
                                pop.lo, pop.hi, pop.c_adh, pop.steps)


@pytest.mark.parametrize("prec", [B.MECH_FP64, B.MECH_FP32_KAHAN, B.MECH_FP32])
def test_noalloc_equals_population_path_twice_second_smaller(prec):
    require_gpu()
    big = workloads.spheroid(20000, seed=4901, steps=30)
    small = _subset(workloads.spheroid(6000, seed=4902, steps=30), 2500, "sph2500")
    for k, (pop, steps) in enumerate(((big, 30), (small, 17))):
        prm = B.params_of(pop, prec)
        say("noalloc", prec, pop.name, steps, "call", k)
        pos, vel, inter = B.step_mechanics_noalloc(prm, pop.pos, pop.radius, pop.type, None, steps)
        wp, wv, wi = _population_path(prm, pop, steps)
        assert np.array_equal(pos, wp) and np.array_equal(vel, wv), (prec, pop.name)
        assert inter == wi


def test_noalloc_history_euler_start_and_untyped_cells():
    require_gpu()
    pop = workloads.plain(1000, seed=1, steps=20)
    vprev = np.random.default_rng(3).normal(0.0, 0.5, (pop.n, 3))
    prm = B.params_of(pop, B.MECH_FP64)
    pos, vel, inter = B.step_mechanics_noalloc(prm, pop.pos, pop.radius, None, vprev, 20)
    wp, wv, wi = _population_path(prm, pop, 20, vprev)
    assert np.array_equal(pos, wp) and np.array_equal(vel, wv) and inter == wi
    prm_e = B.params_of(pop, B.MECH_FP64, ab2_start=B.MECH_AB2_EULER_START)
    pos, vel, inter = B.step_mechanics_noalloc(prm_e, pop.pos, pop.radius, None, None, 5)
    wp, wv, wi = _population_path(prm_e, pop, 5)
    assert np.array_equal(pos, wp) and np.array_equal(vel, wv) and inter == wi


def test_noalloc_zero_steps_empty_and_too_large():
    require_gpu()
    pop = workloads.plain(500, seed=2, steps=0)
    prm = B.params_of(pop, B.MECH_FP64)
    pos, vel, inter = B.step_mechanics_noalloc(prm, pop.pos, pop.radius, None, None, 0)
    wp, wv, wi = _population_path(prm, pop, 0)
    assert np.array_equal(pos, wp) and np.array_equal(vel, wv) and inter == wi == 0
    pos, vel, inter = B.step_mechanics_noalloc(prm, np.zeros((0, 3)), np.zeros(0), None, None, 3)
    assert pos.shape == (0, 3) and inter == 0
    # more cells than the scratch holds: rejected on the host, nothing launched
    big = workloads.tumour(400_000, steps=0)
    with pytest.raises(B.MechError) as e:
        B.step_mechanics_noalloc(B.params_of(big, B.MECH_FP64), big.pos, big.radius, None, None, 1)
    assert e.value.code == B.MECH_E_NOMEM
