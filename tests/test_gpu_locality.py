"""Cells left in their storage order between reorders (the locality study): binning
every step, the candidates read through the sorted index.  The results must be
bitwise those of reordering every step, and the binning still bit-exact."""
import numpy as np
import pytest

import workloads
from gpu_helpers import check_binning, require_gpu, say
from paper_2306_11544_amd import binding as B

pytestmark = pytest.mark.gpu


def _run(pop, prec, steps, every=None):
    prm = B.params_of(pop, prec)
    with B.Population(prm, pop.pos, pop.radius, pop.type) as P:
        if every is not None:
            P.set_reorder(every)
        P.step(steps)
        pos, vel = P.state()
        _, inter, cand = P.stats()
        binning = P.binning()
    return pos, vel, inter, cand, binning


@pytest.mark.parametrize("prec", [B.MECH_FP64, B.MECH_FP32, B.MECH_FP32_KAHAN])
@pytest.mark.parametrize("every", [0, 7])
def test_in_place_steps_equal_reordered_bitwise(prec, every):
    require_gpu()
    pop = workloads.spheroid(20000, seed=61, steps=0)
    say("locality", prec, every)
    ref = _run(pop, prec, 30)
    got = _run(pop, prec, 30, every)
    assert np.array_equal(ref[0], got[0]) and np.array_equal(ref[1], got[1])
    assert ref[2] == got[2] and ref[3] == got[3]


@pytest.mark.parametrize("every", [0, 3])
def test_binning_of_cells_left_in_place_is_exact(orc, every):
    """A step taken in place bins the positions it starts from exactly as the oracle
    bins them (read_binning describes the last step's binning)."""
    require_gpu()
    pop = workloads.spheroid(8000, seed=62, steps=0)
    prm = B.params_of(pop, B.MECH_FP32_KAHAN)
    with B.Population(prm, pop.pos, pop.radius, pop.type) as P:
        P.set_reorder(every)
        P.step(4)             # every = 3: steps 0 and 3 reorder, the fifth is in place
        before, _ = P.state()
        P.step(1)
        vid, start, ids, occ = P.binning()
    want = orc.bin(orc.params_of(pop), before)
    check_binning((vid, start, ids, occ), want, before, pop.lo, pop.hi, pop.voxel)


def test_switching_modes_mid_run():
    """Reorder every step, then never (cells back in id order), then every 5 steps: the
    trajectory is still that of reordering every step."""
    require_gpu()
    pop = workloads.spheroid(6000, seed=63, steps=0)
    prm = B.params_of(pop, B.MECH_FP32_KAHAN)
    ref = _run(pop, B.MECH_FP32_KAHAN, 24)
    with B.Population(prm, pop.pos, pop.radius, pop.type) as P:
        P.step(8)
        P.set_reorder(0)
        P.step(8)
        P.set_reorder(5)
        P.step(8)
        pos, vel = P.state()
    assert np.array_equal(pos, ref[0]) and np.array_equal(vel, ref[1])


def test_negative_interval_rejected():
    require_gpu()
    pop = workloads.plain()
    with B.Population(B.params_of(pop, B.MECH_FP64), pop.pos, pop.radius, pop.type) as P:
        with pytest.raises(B.MechError) as e:
            P.set_reorder(-1)
        assert e.value.code == B.MECH_E_INVALID
