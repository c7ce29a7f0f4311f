"""Binning on the GPU (a1-a5) is bit-exact against the oracle: voxel of every cell, voxel
starts, occupied list, and the cells of each voxel; the order inside a voxel is checked
against the library's documented storage order.

Compared at creation, where both sides bin the same seeded positions: the three
single-simulation workloads at full size (1k, 100k, 1M cells), positions the oracle
evolved for many steps, adversarial positions on voxel faces and walls, a pile of
cells in one voxel, and degenerate grids."""
import numpy as np
import pytest

import workloads
from gpu_helpers import check_binning, require_gpu, say
from paper_2306_11544_amd import binding as B

pytestmark = pytest.mark.gpu


def _compare(orc, pop, precision=B.MECH_FP64):
    say("binning", pop.name, pop.n, precision)
    want = orc.bin(orc.params_of(pop), pop.pos)
    with B.Population(B.params_of(pop, precision), pop.pos, pop.radius, pop.type) as P:
        got = P.binning()
    check_binning(got, want, pop.pos, pop.lo, pop.hi, pop.voxel)


@pytest.mark.parametrize("name", ["plain1k", "sph100k", "tumour1m"])
def test_binning_full_size(orc, name):
    require_gpu()
    _compare(orc, workloads.config(name))


def test_binning_fp32_state(orc):
    require_gpu()
    _compare(orc, workloads.spheroid(30000, seed=5), B.MECH_FP32_KAHAN)


def test_binning_after_oracle_steps(orc):
    require_gpu()
    pop = workloads.spheroid(20000, seed=6)
    evolved = orc.run_pop(pop, steps=200)["pos"]
    pop.pos = evolved
    _compare(orc, pop)


def test_binning_adversarial_faces(orc):
    require_gpu()
    pop = workloads.plain(5000, seed=7)
    rng = np.random.default_rng(8)
    faces = -100.0 + 30.0 * np.arange(7)
    vals = np.concatenate([faces, np.nextafter(faces, np.inf), np.nextafter(faces, -np.inf),
                           [-100.0, 100.0, -0.0, 0.0, np.nextafter(100.0, -np.inf)]])
    vals = vals[(vals >= -100.0) & (vals <= 100.0)]
    pop.pos = rng.choice(vals, size=(pop.n, 3))
    _compare(orc, pop)


def test_binning_pile_in_one_voxel(orc):
    require_gpu()
    pop = workloads.plain(3000, seed=9)
    rng = np.random.default_rng(10)
    pop.pos = 5.0 + rng.uniform(0, 1e-3, size=(pop.n, 3))
    _compare(orc, pop)


def test_binning_flat_domain(orc):
    require_gpu()
    pop = workloads.plain(2000, seed=11)
    pop.lo = (pop.lo[0], pop.lo[1], 0.0)
    pop.hi = (pop.hi[0], pop.hi[1], 0.0)
    pop.pos[:, 2] = 0.0
    _compare(orc, pop)


def test_binning_ragged_sizes(orc):
    require_gpu()
    for n in (1, 2, 63, 65, 255, 257, 4097):
        _compare(orc, workloads.spheroid(n, seed=100 + n))


def test_binning_large_grid_scan_path(orc):
    """A grid of more than 2048 scan tiles (4 bins per voxel, 2048 bins per tile: above
    1,048,576 voxels) takes the separate tile-sum scan (k_scan_top) instead of the fused
    one; its output is compared bit for bit too.  A sparse 3.3 mm cube: 110^3 = 1,331,000
    voxels for 200,000 cells."""
    require_gpu()
    pop = workloads.plain(200_000, seed=12, half=1650.0)
    assert np.prod(orc.grid_dims(orc.params_of(pop))) * 4 > 2048 * 2048
    _compare(orc, pop)
