"""The force kernel's candidate pruning against geometry built to sit on its edges: the
prefilter (quantised shadow, integer test) and the slab window must drop no pair that
the exact decision counts.  Pairs sit at the repulsion and adhesion cutoffs to a
relative 1e-6 .. 1e-15 on either side; one domain lies far from the origin, where the
quantised coordinates wrap their 16 bits many times over and float positions keep few
bits below the micrometre; the voxel is the smallest allowed (h = 2 alpha r_max, the
widest reach per voxel).  The list kernel, at every list length and trip size, must give
the inline kernel's interaction counts and trajectories bitwise; the inline kernel
evaluates every pair of the 27 voxels."""
import numpy as np
import pytest

import workloads
from gpu_helpers import require_gpu, say
from paper_2306_11544_amd import binding as B

pytestmark = pytest.mark.gpu

ALPHA = 1.25
R_MAX = 10.0
H = 2 * ALPHA * R_MAX          # the smallest voxel the library accepts for R_MAX


def _edge_population(seed, lo0):
    rng = np.random.default_rng(seed)
    side = 8 * H
    lo = np.asarray(lo0, np.float64)
    hi = lo + side
    n_bg = 1200
    pos = [lo + rng.uniform(0.05, 0.95, (n_bg, 3)) * side]
    rad = [rng.uniform(5.0, R_MAX, n_bg)]
    rad[0][0] = R_MAX
    rels = (1e-6, 1e-9, 1e-12, 1e-15, 0.0, -1e-15, -1e-12, -1e-9, -1e-6)
    for _ in range(12):
        r1, r2 = rng.uniform(5.0, R_MAX, 2)
        for target in (r1 + r2, ALPHA * (r1 + r2)):
            for rel in rels:
                s = target * (1.0 + rel)
                u = rng.normal(size=3)
                u /= np.linalg.norm(u)
                c = lo + rng.uniform(0.1, 0.9, 3) * side
                pos.append(np.stack([c - 0.5 * s * u, c + 0.5 * s * u]))
                rad.append(np.array([r1, r2]))
    pos = np.concatenate(pos)
    rad = np.concatenate(rad)
    typ = rng.integers(0, 2, len(rad)).astype(np.int32)
    return workloads.Population(name=f"edge{seed}", pos=pos, radius=rad, type=typ, lo=tuple(lo),
                                hi=tuple(hi), c_adh=workloads.C_ADH_2, steps=5, voxel=H)


def _run(pops, tuning, steps, prec):
    p = B.make_params((0, 0, 0), (1, 1, 1), voxel_size=H, rel_adh_distance=ALPHA,
                      c_adh=workloads.C_ADH_2, precision=prec)
    cells = sum(x.n for x in pops)
    vox = sum(B.batch_request_voxels(p, x.lo, x.hi) for x in pops)
    with B.Batch(p, cells, vox, len(pops)) as bt:
        bt.set_tuning(tuning)
        slots = [bt.admit_pop(x, n_steps=steps) for x in pops]
        bt.step(1)
        _, inter1, _ = bt.stats()
        bt.step(steps - 1)
        res = [bt.read(s) for s in slots]
    return res, inter1


@pytest.mark.parametrize("prec", [B.MECH_FP64, B.MECH_FP32, B.MECH_FP32_KAHAN])
def test_prefilter_keeps_every_edge_pair(prec):
    require_gpu()
    pops = [_edge_population(71, (0.0, 0.0, 0.0)),
            _edge_population(72, (-37011.3, 52000.7, 100000.1))]
    ref, inter_ref = _run(pops, B.tuning("rows", 4, 4, 0), 5, prec)
    assert inter_ref > 0
    for cfg in [("cells", 4, 4, 0, 16), ("cells", 1, 8, 0, 16), ("cells", 2, 2, 0, 16),
                ("cells", 4, 4, 0, 32), ("cells", 1, 8, 0, 64)]:
        say("prefilter edges", prec, cfg)
        got, inter = _run(pops, B.tuning(*cfg), 5, prec)
        assert inter == inter_ref, cfg
        for (p0, v0), (p1, v1) in zip(ref, got):
            assert np.array_equal(p0, p1) and np.array_equal(v0, v1), cfg


def test_edge_pairs_are_counted_as_the_oracle_counts(orc):
    """FP64 first-step interaction count of the far domain equals the oracle's."""
    require_gpu()
    pop = _edge_population(72, (-37011.3, 52000.7, 100000.1))
    _, inter = _run([pop], B.tuning("cells", 4, 4, 0, 16), 1, B.MECH_FP64)
    p = orc.params(pop.lo, pop.hi, h=H, alpha=ALPHA, c_adh=workloads.C_ADH_2)
    _, want, _ = orc.velocity_voxel(p, pop.pos, pop.radius, pop.type, orc.FP64)
    assert inter == want
