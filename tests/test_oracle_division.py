"""Pins of the division rule of growing populations (oracle side).

The draws are SplitMix64 outputs; its published reference sequence (state 0, three
steps) fixes the generator.  The rule itself is checked on cases where every
quantity is known: with no forces a cell stays put through the step, so parent and
daughter must sit at distance r around it, with ids, radii and types as defined."""
import os

import numpy as np
import pytest

import workloads

GOLDEN = 0x9E3779B97F4A7C15
M64 = (1 << 64) - 1


def test_splitmix64_reference_sequence(orc):
    # the generator's published outputs from state 0 (tests/golden): next() adds the
    # golden gamma to the state and returns the mixed value
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                        "splitmix64_reference.txt")
    want = [int(line, 16) for line in open(path) if line.strip() and not line.startswith("#")]
    assert len(want) == 3
    got = [orc.splitmix64((GOLDEN * k) & M64) for k in (1, 2, 3)]
    assert got == want


def test_uniform_draws_are_uniform(orc):
    u = np.array([orc.uniform(7, i, 3, 0) for i in range(20000)])
    assert u.min() >= 0.0 and u.max() < 1.0
    assert abs(u.mean() - 0.5) < 0.01
    assert abs((u < 0.1).mean() - 0.1) < 0.01
    # distinct counters give distinct draws
    assert len({orc.uniform(7, 5, t, k) for t in range(20) for k in range(4)}) == 80


def _still(orc, pop):
    """Parameters with no forces: integration leaves every cell where it is."""
    return orc.params(pop.lo, pop.hi, h=pop.voxel, dt=pop.dt, c_rep=0.0, alpha=pop.alpha,
                      c_adh=((0.0,),))


def test_every_cell_divides_around_its_position(orc):
    pop = workloads.plain(200, seed=11)
    pos = np.clip(pop.pos, -80, 80)   # away from the walls
    types = (np.arange(pop.n) % 2).astype(np.int32)
    r = orc.run_growing(_still(orc, pop), pos, pop.radius, types, steps=1, capacity=2 * pop.n,
                        p_div=1.0, seed=3)
    n = pop.n
    assert r["n"] == 2 * n
    parent, daughter = r["pos"][:n], r["pos"][n:]
    np.testing.assert_allclose(np.linalg.norm(daughter - parent, axis=1), pop.radius, rtol=1e-12)
    np.testing.assert_allclose((daughter + parent) / 2, pos, atol=1e-12)
    assert np.array_equal(r["radius"][n:], pop.radius)
    assert np.array_equal(r["type"][n:], types)


def test_division_draws_select_cells_and_rank_daughters(orc):
    pop = workloads.plain(500, seed=12)
    pos = np.clip(pop.pos, -80, 80)
    p_div, seed = 0.2, 9
    r = orc.run_growing(_still(orc, pop), pos, pop.radius, steps=1, capacity=2 * pop.n,
                        p_div=p_div, seed=seed)
    chosen = [i for i in range(pop.n) if orc.uniform(seed, i, 0, 0) < p_div]
    assert r["n"] == pop.n + len(chosen)
    for k, i in enumerate(chosen):   # daughter of rank k has id n + k
        d = r["pos"][pop.n + k] - pos[i]
        assert abs(np.linalg.norm(d) - pop.radius[i] / 2) < 1e-12
    unchanged = np.setdiff1d(np.arange(pop.n), chosen)
    assert np.array_equal(r["pos"][unchanged], pos[unchanged])


def test_capacity_limits_division_by_id(orc):
    pop = workloads.plain(100, seed=13)
    pos = np.clip(pop.pos, -80, 80)
    r = orc.run_growing(_still(orc, pop), pos, pop.radius, steps=1, capacity=pop.n + 3,
                        p_div=1.0, seed=1)
    assert r["n"] == pop.n + 3
    moved = np.flatnonzero(np.any(r["pos"][:pop.n] != pos, axis=1))
    assert list(moved) == [0, 1, 2]


def test_no_division_is_the_plain_method(orc):
    pop = workloads.plain()
    p = orc.params_of(pop)
    a = orc.run_growing(p, pop.pos, pop.radius, steps=20, capacity=pop.n, p_div=0.0)
    b = orc.run(p, pop.pos, pop.radius, pop.type, steps=20)
    assert np.array_equal(a["pos"], b["pos"])
    assert a["interactions"] == b["interactions"]


def test_daughters_stay_in_the_domain(orc):
    pop = workloads.plain(300, seed=14)
    pos = pop.pos.copy()
    pos[:50, 0] = 100.0   # on the upper wall
    r = orc.run_growing(_still(orc, pop), pos, pop.radius, steps=1, capacity=2 * pop.n,
                        p_div=1.0, seed=2)
    assert r["pos"].min() >= -100.0 and r["pos"].max() <= 100.0
