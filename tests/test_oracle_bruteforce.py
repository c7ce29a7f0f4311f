"""Pins the 27-voxel search against the plain O(n^2) definition on small inputs.

With a voxel edge h >= 1.25 (r_i + r_j) for every pair, every interacting pair lies in
the 27 voxels around the cell, so the voxel method must find exactly the same pairs
(equal integer counts) and the same velocities up to summation order.  Inputs cover
the three single-simulation workload geometries at a size the O(n^2) loop finishes in
well under a second, cells on walls, two types, and radii at the clip bounds.
"""
import numpy as np
import pytest

import workloads


def _cases():
    yield "plain1k", workloads.plain()
    yield "sph2k", workloads.spheroid(2000, seed=7)
    # tumour geometry scaled so that 2000 cells keep the 1M-cell core density
    f = (2000 / 1e6) ** (1 / 3)
    yield "tumour2k", workloads.tumour(2000, seed=8, core_radius=600 * f, half=1000 * f)
    pop = workloads.spheroid(1500, seed=9)
    pop.radius[::2] = 6.0
    pop.radius[1::2] = 11.0
    yield "clip_radii", pop
    # cells pressed onto walls and corners
    pop = workloads.plain(800, seed=10, half=45.0)
    pop.pos[:100, 0] = pop.hi[0]
    pop.pos[100:200, 1] = pop.lo[1]
    pop.pos[200:210] = np.array(pop.hi)
    yield "walls", pop


CASES = list(_cases())


@pytest.mark.parametrize("name,pop", CASES, ids=[c[0] for c in CASES])
def test_voxel_equals_allpairs_fp64(orc, name, pop):
    p = orc.params_of(pop)
    va, ia = orc.velocity_allpairs(p, pop.pos, pop.radius, pop.type)
    vv, iv, cand = orc.velocity_voxel(p, pop.pos, pop.radius, pop.type)
    assert ia == iv and ia > 0
    assert cand >= iv
    scale = np.abs(va).max()
    assert np.abs(va - vv).max() <= 1e-13 * max(scale, 1.0)


@pytest.mark.parametrize("precision", [1, 2])
@pytest.mark.parametrize("name,pop", CASES[:3], ids=[c[0] for c in CASES[:3]])
def test_voxel_equals_allpairs_fp32(orc, name, pop, precision):
    p = orc.params_of(pop)
    va, ia = orc.velocity_allpairs(p, pop.pos, pop.radius, pop.type, precision)
    vv, iv, _ = orc.velocity_voxel(p, pop.pos, pop.radius, pop.type, precision)
    assert ia == iv  # the float decisions are the same on both sides
    scale = np.abs(va).max()
    assert np.abs(va - vv).max() <= 2e-5 * scale


@pytest.mark.parametrize("name,pop", CASES[:3], ids=[c[0] for c in CASES[:3]])
def test_fp32_close_to_fp64(orc, name, pop):
    p = orc.params_of(pop)
    v64, i64, _ = orc.velocity_voxel(p, pop.pos, pop.radius, pop.type, 0)
    v32, i32, _ = orc.velocity_voxel(p, pop.pos, pop.radius, pop.type, 2)
    # a float decision can only differ for a pair within float rounding of its cutoff
    assert abs(i64 - i32) <= 2
    assert np.abs(v64 - v32).max() <= 1e-4 * np.abs(v64).max()


def test_per_step_interactions_all_pairs_trajectory(orc):
    pop = workloads.spheroid(1000, seed=13)
    p = orc.params_of(pop)
    a = orc.run(p, pop.pos, pop.radius, pop.type, steps=30, per_step=True)
    b = orc.run(p, pop.pos, pop.radius, pop.type, steps=30, allpairs=True, per_step=True)
    assert np.array_equal(a["per_step_interactions"], b["per_step_interactions"])
    assert np.abs(a["pos"] - b["pos"]).max() < 1e-12 * pop.half_width


def test_sampled_velocity_matches_full(orc):
    pop = workloads.spheroid(5000, seed=14)
    p = orc.params_of(pop)
    ids = np.array([0, 7, 4999, 2500, 1234])
    for prec in (0, 2):
        v, _, _ = orc.velocity_voxel(p, pop.pos, pop.radius, pop.type, prec)
        vs, _ = orc.velocity_sampled(p, pop.pos, pop.radius, pop.type, ids, prec)
        assert np.array_equal(v[ids], vs)
