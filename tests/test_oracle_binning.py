"""Pins the oracle's binning against numpy floor + lexsort (a library routine).

Binning is integer work and must be bit-exact: voxel of each cell, the exclusive
prefix of voxel counts, cells ordered by (voxel, id) -- a counting sort by voxel that is
stable in cell id -- and the list of occupied voxels.
Adversarial positions sit exactly on voxel and slab faces, on lo and hi, one ulp
either side of a face, and at -0.0.
"""
import numpy as np
import pytest

import workloads


def numpy_bin(lo, hi, h, pos):
    lo = np.asarray(lo, float)
    dims = np.maximum(1, np.ceil((np.asarray(hi, float) - lo) / h)).astype(np.int64)
    k = np.floor((pos - lo) * (1.0 / h))
    k = np.clip(k, 0, dims - 1).astype(np.int64)
    vid = k[:, 0] + dims[0] * (k[:, 1] + dims[1] * k[:, 2])
    V = int(np.prod(dims))
    order = np.lexsort((np.arange(len(pos)), vid))
    start = np.concatenate([[0], np.cumsum(np.bincount(vid, minlength=V))])
    occ = np.unique(vid)
    return vid.astype(np.uint32), start.astype(np.uint32), order.astype(np.uint32), occ.astype(np.uint32)


def adversarial(n=4000, seed=3):
    lo, hi, h = (-100.0,) * 3, (100.0,) * 3, 30.0
    rng = np.random.default_rng(seed)
    faces = -100.0 + (h / 4) * np.arange(0, 29)   # voxel and slab faces
    faces = faces[faces <= 100.0]
    vals = np.concatenate([faces, np.nextafter(faces, np.inf), np.nextafter(faces, -np.inf),
                           [-100.0, 100.0, -0.0, 0.0, np.nextafter(100.0, -np.inf)]])
    vals = vals[(vals >= -100.0) & (vals <= 100.0)]
    pos = rng.choice(vals, size=(n, 3))
    pos[: n // 4] = rng.uniform(-100, 100, size=(n // 4, 3))
    return lo, hi, h, pos


def _cases():
    for name, pop in (("plain1k", workloads.plain()), ("sph20k", workloads.spheroid(20000, seed=2)),
                      ("tumour20k", workloads.tumour(20000, seed=3))):
        yield name, pop.lo, pop.hi, pop.voxel, pop.pos
    yield ("adversarial",) + adversarial()
    # grid that overruns hi (7 * 30 = 210 > 200) and a domain that is a whole number
    lo, hi, h, pos = adversarial(2000, seed=4)
    yield "whole_voxels", (-90.0,) * 3, (90.0,) * 3, 30.0, np.clip(pos, -90, 90)
    yield "empty", (-100.0,) * 3, (100.0,) * 3, 30.0, np.zeros((0, 3))
    yield "one_voxel_pile", (-100.0,) * 3, (100.0,) * 3, 30.0, np.full((300, 3), 5.0)


CASES = list(_cases())


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_binning_matches_numpy(orc, case):
    name, lo, hi, h, pos = case
    p = orc.params(lo, hi, h=h)
    got = orc.bin(p, pos)
    want = numpy_bin(lo, hi, h, pos)
    for g, w in zip(got, want):
        assert g.dtype == np.uint32
        assert np.array_equal(g, w)


def test_voxel_numbering_is_x_fastest(orc):
    p = orc.params((0.0,) * 3, (90.0,) * 3, h=30.0)
    pos = np.array([[31.0, 1.0, 1.0], [1.0, 31.0, 1.0], [1.0, 1.0, 31.0], [89.0, 89.0, 89.0]])
    vid, _, _, _ = orc.bin(p, pos)
    assert list(vid) == [1, 3, 9, 26]


def test_ties_broken_by_ascending_id(orc):
    """Cells of one voxel are listed by ascending id, wherever they sit in it."""
    p = orc.params((0.0,) * 3, (90.0,) * 3, h=30.0)
    x = np.array([29.0, 1.0, 16.0, 7.5, 7.4999, 22.5, 0.0, 15.0, 45.0, 31.0])
    pos = np.stack([x, np.full_like(x, 3.0), np.full_like(x, 3.0)], axis=1)
    vid, start, order, occ = orc.bin(p, pos)
    assert list(vid) == [0] * 8 + [1, 1]
    assert list(order) == [0, 1, 2, 3, 4, 5, 6, 7, 8, 9]
    assert list(start[:3]) == [0, 8, 10] and list(occ) == [0, 1]
