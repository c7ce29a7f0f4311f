"""Pins the oracle with properties the mechanics must have at any size.

Newton's third law (pair terms are antisymmetric, so the velocities sum to zero up to
rounding), a fixed centre of mass away from the walls, invariance under translation of
cells and domain together and under a relabelling of cells, an isolated cell at rest,
a symmetric lattice whose centre feels no net force, and reflecting walls worked out by
hand on prescribed velocities.
"""
import numpy as np
import pytest

import workloads


def _pop_params(orc, pop):
    return orc.params_of(pop)


@pytest.mark.parametrize("maker", [lambda: workloads.plain(),
                                   lambda: workloads.spheroid(3000, seed=11),
                                   lambda: workloads.tumour(3000, seed=12, core_radius=82.0,
                                                            half=130.0)])
@pytest.mark.parametrize("precision", [0, 2])
def test_newton_third_law(orc, maker, precision):
    pop = maker()
    p = _pop_params(orc, pop)
    v, inter, _ = orc.velocity_voxel(p, pop.pos, pop.radius, pop.type, precision)
    assert inter > 0
    scale = np.abs(v).sum()
    tol = 1e-13 if precision == 0 else 1e-6
    assert np.abs(v.sum(axis=0)).max() <= tol * scale


def test_centre_of_mass_fixed_away_from_walls(orc):
    pop = workloads.spheroid(400, seed=21, two_types=True)
    # put the ball in a domain far larger than it, so that no cell reaches a wall
    p = orc.params((-600.0,) * 3, (600.0,) * 3, c_adh=pop.c_adh)
    out = orc.run(p, pop.pos, pop.radius, pop.type, steps=60)
    moved = np.abs(out["pos"] - pop.pos).max()
    assert moved > 0.5
    assert np.abs(out["pos"].mean(axis=0) - pop.pos.mean(axis=0)).max() < 1e-12


def test_translation_invariance(orc):
    pop = workloads.plain()
    shift = np.array([17.3, -41.1, 90.0])  # not a multiple of the voxel edge
    p0 = orc.params_of(pop)
    p1 = orc.params(np.array(pop.lo) + shift, np.array(pop.hi) + shift, c_adh=pop.c_adh)
    a = orc.run(p0, pop.pos, pop.radius, pop.type, steps=100)["pos"]
    b = orc.run(p1, pop.pos + shift, pop.radius, pop.type, steps=100)["pos"] - shift
    assert np.abs(a - b).max() <= 1e-11 * pop.half_width


def test_permutation_invariance(orc):
    pop = workloads.spheroid(2000, seed=31)
    p = orc.params_of(pop)
    perm = np.random.default_rng(5).permutation(pop.n)
    a = orc.run(p, pop.pos, pop.radius, pop.type, steps=20)
    b = orc.run(p, pop.pos[perm], pop.radius[perm], pop.type[perm], steps=20)
    assert a["interactions"] == b["interactions"]
    assert np.abs(a["pos"][perm] - b["pos"]).max() < 1e-13 * pop.half_width * 100


def test_isolated_cell_at_rest(orc):
    p = orc.params((-100.0,) * 3, (100.0,) * 3)
    pos = np.array([[3.0, -4.0, 5.0], [60.0, 60.0, 60.0]])
    out = orc.run(p, pos, np.array([8.4, 11.0]), steps=50)
    assert np.array_equal(out["pos"], pos)
    assert out["interactions"] == 0


def test_symmetric_lattice_centre(orc):
    # spacing 14 um: edge neighbours repel, face diagonals (19.8 um) adhere,
    # body diagonals (24.2 um) are out of reach
    g = np.arange(-1, 2) * 14.0
    pos = np.array([[x, y, z] for z in g for y in g for x in g])
    p = orc.params((-100.0,) * 3, (100.0,) * 3)
    v, inter, _ = orc.velocity_voxel(p, pos, np.full(len(pos), 8.4))
    centre = 13
    assert np.abs(v[centre]).max() < 1e-14
    assert np.abs(v[0]).max() > 1e-3          # corners do feel a force
    # by symmetry the corner velocity points along the body diagonal
    assert np.allclose(v[0] / np.linalg.norm(v[0]), -np.ones(3) / np.sqrt(3), atol=1e-12)


def test_voxel_smaller_than_reach_misses_pairs(orc):
    """Why h must cover the longest adhesion reach 2.5 r_max: with h = 15 um the 27-voxel
    search misses pairs that the all-pairs definition finds."""
    pop = workloads.spheroid(1500, seed=41)
    p_small = orc.params(pop.lo, pop.hi, h=15.0, c_adh=pop.c_adh)
    _, i_all = orc.velocity_allpairs(p_small, pop.pos, pop.radius, pop.type)
    _, i_vox, _ = orc.velocity_voxel(p_small, pop.pos, pop.radius, pop.type)
    assert i_vox < i_all


# ----------------------------------------------------------------- integration + walls

def _integrate(orc, x, v, vp, euler=False, lo=-100.0, hi=100.0, dt=0.1):
    p = orc.params((lo,) * 3, (hi,) * 3, dt=dt)
    pos = np.array([x], dtype=np.float64)
    vprev = np.array([vp], dtype=np.float64)
    orc.integrate(p, pos, np.array([v], dtype=np.float64), vprev, euler)
    return pos[0], vprev[0]


def test_ab2_update_and_history(orc):
    x, vp = _integrate(orc, [1.0, 2.0, 3.0], [1.0, -2.0, 0.5], [4.0, 0.0, -1.0])
    # x + dt (1.5 v - 0.5 v_prev)
    assert np.allclose(x, [1.0 + 0.1 * (1.5 - 2.0), 2.0 + 0.1 * (-3.0), 3.0 + 0.1 * (0.75 + 0.5)],
                       rtol=0, atol=1e-15)
    assert np.array_equal(vp, [1.0, -2.0, 0.5])


def test_euler_start_ignores_history(orc):
    x, _ = _integrate(orc, [1.0, 2.0, 3.0], [1.0, -2.0, 0.5], [4.0, 7.0, -1.0], euler=True)
    assert np.allclose(x, [1.1, 1.8, 3.05], rtol=0, atol=1e-15)


def test_reflecting_wall_high_and_low(orc):
    # x = hi - 0.5 moving +10 um/min with no history: 1.5 dt v = 1.5 um -> hi + 1.0 -> hi - 1.0
    x, _ = _integrate(orc, [99.5, -99.5, 0.0], [10.0, -10.0, 0.0], [0.0, 0.0, 0.0])
    assert np.allclose(x, [99.0, -99.0, 0.0], rtol=0, atol=1e-13)


def test_reflection_overshoot_is_clamped(orc):
    # x: 99.5 + 1500 = 1599.5 -> mirrored at hi to -1399.5 -> clamped to lo
    # y: -99.5 - 1500 = -1599.5 -> mirrored at lo to 1399.5 -> mirrored at hi to -1199.5
    #    -> clamped to lo
    x, vp = _integrate(orc, [99.5, -99.5, 50.0], [10000.0, -10000.0, 0.0], [0.0, 0.0, 0.0])
    assert np.array_equal(x, [-100.0, -100.0, 50.0])
    assert np.array_equal(vp, [10000.0, -10000.0, 0.0])  # history is not reflected


def test_cell_on_the_wall_stays_in_domain(orc):
    x, _ = _integrate(orc, [100.0, -100.0, 100.0], [0.0, 0.0, 1e-3], [0.0, 0.0, 0.0])
    assert np.all(x <= 100.0) and np.all(x >= -100.0)
