"""Pins of the death rule of dynamic populations (oracle side).

The death draw is recomputed here from the SplitMix64 definition (written out below,
independent of the oracle's C code); with no forces every cell stays put through the
step, so the survivors' state must equal their state before it, in id order."""
import numpy as np

import workloads

GOLDEN = 0x9E3779B97F4A7C15
M64 = (1 << 64) - 1


def _splitmix64(state):
    z = state & M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M64
    return z ^ (z >> 31)


def _uniform(seed, cell_id, t, k):
    counter = 4 * ((t << 32) + cell_id) + k + 1
    return (_splitmix64(seed + GOLDEN * counter) >> 11) * 2.0 ** -53


def _death(seed, cell_id, t):
    return _uniform(seed ^ (1 << 63), cell_id, t, 0)


def _still(orc, pop):
    return orc.params(pop.lo, pop.hi, h=pop.voxel, dt=pop.dt, c_rep=0.0, alpha=pop.alpha,
                      c_adh=((0.0,),))


def test_death_draw_is_the_flipped_seed_stream(orc):
    for seed, cid, t in [(0, 0, 0), (3, 17, 5), (2**63 + 5, 999, 123), (M64, 2**31 - 1, 7)]:
        assert orc.death_draw(seed, cid, t) == _death(seed, cid, t)
        assert orc.uniform(seed, cid, t, 0) == _uniform(seed, cid, t, 0)


def test_death_and_division_streams_differ(orc):
    same = sum(orc.death_draw(5, i, t) == orc.uniform(5, i, t, 0) for i in range(300) for t in range(5))
    assert same == 0


def test_survivors_are_the_cells_whose_draw_passes(orc):
    pop = workloads.plain(400, seed=21)
    types = (np.arange(pop.n) % 3 == 0).astype(np.int32)
    p_death, seed = 0.3, 77
    r = orc.run_growing(_still(orc, pop), pop.pos, pop.radius, types, steps=1, seed=seed,
                        p_death=p_death)
    keep = [i for i in range(pop.n) if not (_death(seed, i, 0) < p_death)]
    assert 0 < len(keep) < pop.n
    assert r["n"] == len(keep) == r["per_step_n"][0]
    np.testing.assert_array_equal(r["pos"], pop.pos[keep])
    np.testing.assert_array_equal(r["radius"], pop.radius[keep])
    np.testing.assert_array_equal(r["type"], types[keep])


def test_no_death_and_certain_death(orc):
    pop = workloads.plain(300, seed=22)
    p = orc.params_of(pop)
    a = orc.run_growing(p, pop.pos, pop.radius, steps=5, seed=1, p_death=0.0)
    b = orc.run_growing(p, pop.pos, pop.radius, steps=5)
    np.testing.assert_array_equal(a["pos"], b["pos"])
    c = orc.run_growing(p, pop.pos, pop.radius, steps=2, seed=1, p_death=1.0)
    assert c["n"] == 0 and c["per_step_n"] == [0, 0]


def test_death_follows_division_and_takes_daughters_too(orc):
    pop = workloads.plain(300, seed=23)
    pos = np.clip(pop.pos, -80, 80)
    p_div, p_death, seed = 0.4, 0.25, 9
    r = orc.run_growing(_still(orc, pop), pos, pop.radius, steps=1, capacity=2 * pop.n,
                        p_div=p_div, p_death=p_death, seed=seed)
    n = pop.n
    made = sum(_uniform(seed, i, 0, 0) < p_div for i in range(n))
    grown = n + made
    keep = [i for i in range(grown) if not (_death(seed, i, 0) < p_death)]
    assert r["n"] == len(keep)
    # dead daughters and parents both leave; the survivors' radii follow id order
    radius = np.concatenate([pop.radius, pop.radius[[i for i in range(n) if _uniform(seed, i, 0, 0) < p_div]]])
    np.testing.assert_array_equal(r["radius"], radius[keep])
