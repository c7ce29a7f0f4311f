"""With exactly two cell types the FP32 kernels take a candidate's type from the sign of
the float shadow's radius, and read no type array.  Declaring a third, unused type (the
same adhesion coefficients for types 0 and 1) sends the same cells through the kernels
that read the type array: positions, velocities and the exact counts must be equal bit
for bit.  Each of the three writers of the shadow is covered: the gather of a large
population, the one-workgroup binning of a small one, and the shadow kernel of cells
left in place between reorders."""
import numpy as np
import pytest

import workloads
from gpu_helpers import require_gpu, say
from paper_2306_11544_amd import binding as B

pytestmark = pytest.mark.gpu

# types 0 and 1 as in the two-type workloads, and a third type no cell has
C_ADH_3 = [[0.4, 0.1, 0.25], [0.1, 0.4, 0.3], [0.25, 0.3, 0.4]]


def _run(pop, c_adh, prec, steps, reorder_every):
    p = B.make_params(pop.lo, pop.hi, pop.voxel, pop.dt, pop.c_rep, pop.alpha, c_adh, prec)
    with B.Population(p, pop.pos, pop.radius, pop.type) as P:
        P.set_reorder(reorder_every)
        P.step(steps)
        pos, vel = P.state()
        _, inter, cand = P.stats()
    return pos, vel, inter, cand


@pytest.mark.parametrize("prec", [B.MECH_FP32, B.MECH_FP32_KAHAN])
@pytest.mark.parametrize("n,reorder_every", [(20_000, 1), (5_000, 1), (20_000, 0)],
                         ids=["gather", "small-population", "in-place"])
def test_sign_typed_shadow_equals_type_array(prec, n, reorder_every):
    require_gpu()
    pop = workloads.spheroid(n, seed=78, steps=0)
    assert np.array_equal(np.unique(pop.type), [0, 1])
    assert np.array_equal(np.asarray(C_ADH_3)[:2, :2], workloads.C_ADH_2)
    say("shadow type", n, "cells, precision", prec, "reorder every", reorder_every)
    two = _run(pop, workloads.C_ADH_2, prec, 40, reorder_every)
    three = _run(pop, C_ADH_3, prec, 40, reorder_every)
    assert two[2] > 0
    assert np.array_equal(two[0], three[0])
    assert np.array_equal(two[1], three[1])
    assert two[2:] == three[2:]
