"""Shared helpers of the GPU parity tests (not collected: no test_ prefix)."""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

from paper_2306_11544_amd import binding as B


def say(*a):
    """Name the case before a GPU step, flushed, so a crash log points at it."""
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


def require_gpu():
    n = B.mech_device_count()
    assert n > 0, "no HIP device visible to libmech.so"


def run_gpu(pop, steps, precision=B.MECH_FP64, ab2_start=B.MECH_AB2_ZERO_HISTORY, flags=0,
            per_step=False, prev_velocity=None):
    """Run `steps` steps; returns dict(pos, vel, interactions, candidates[, per_step])."""
    p = B.params_of(pop, precision, ab2_start, flags)
    with B.Population(p, pop.pos, pop.radius, pop.type, prev_velocity) as P:
        per = []
        if per_step:
            last = 0
            for _ in range(steps):
                P.step(1)
                _, it, _ = P.stats()
                per.append(it - last)
                last = it
        else:
            P.step(steps)
        pos, vel = P.state()
        s, it, cand = P.stats()
        assert s == steps
    out = dict(pos=pos, vel=vel, interactions=it, candidates=cand)
    if per_step:
        out["per_step"] = np.array(per, dtype=np.int64)
    return out


def record(case, err, **extra):
    """Append a parity error to the JSON-lines file named by MECH_PARITY_LOG, if set:
    the per-configuration error table is collected this way."""
    out = os.environ.get("MECH_PARITY_LOG")
    if out and os.path.isdir(os.path.dirname(os.path.abspath(out))):
        with open(out, "a") as f:
            f.write(json.dumps({"case": case, "err": float(err), **extra}) + "\n")


def assert_well_posed(orc, pop, steps, bar=1e-10):
    """The oracle's own trajectory moves by far less than the bar when every input
    coordinate is nudged by one ulp, and when the cells are relabelled (which changes
    the order of every force sum).  Otherwise the case is chaotic at this horizon and
    no implementation that sums in another order could be held to the bar."""
    p = orc.params_of(pop)
    a = orc.run(p, pop.pos, pop.radius, pop.type, steps=steps)["pos"]
    b = orc.run(p, np.nextafter(pop.pos, 0.0), pop.radius, pop.type, steps=steps)["pos"]
    perm = np.random.default_rng(0).permutation(pop.n)
    c = np.empty_like(a)
    c[perm] = orc.run(p, pop.pos[perm], pop.radius[perm], pop.type[perm], steps=steps)["pos"]
    sens = max(pos_err(a, b, pop.half_width), pos_err(a, c, pop.half_width))
    assert sens <= bar / 100, f"ill-posed case: sensitivity {sens:.2e}"


def disp_err(got, want, x0):
    """Displacement-relative error: |(x_gpu - x0) - (x_oracle - x0)| / |x_oracle - x0|, the
    norms taken over all cells and axes; the error measured against how far the cells
    moved from their start x0 (0 when they did not move)."""
    d = np.linalg.norm(np.asarray(want) - np.asarray(x0))
    return float(np.linalg.norm(np.asarray(got) - np.asarray(want)) / d) if d > 0 else 0.0


def pos_err(a, b, S):
    """Domain-scaled position error: max over cells and axes of |a - b| / S."""
    if a.size == 0:
        return 0.0
    return float(np.abs(a - b).max() / S)


def storage_order(pos, lo, hi, h):
    """The order the library stores cells in, computed with numpy: by voxel, then by x slab
    (the voxel cut in four along x, slab floor((x - lo) * (1/h) * 4) - 4 kx, clamped like
    the voxel index), then by id.  The voxel and the ids inside it are the method's; the
    slab order is the library's own choice (it keeps a neighbour row's cells within reach
    of a cell along x contiguous), so it is checked here and not by the oracle."""
    pos = np.asarray(pos, dtype=np.float64).reshape(-1, 3)
    lo = np.asarray(lo, float)
    dims = np.maximum(1, np.ceil((np.asarray(hi, float) - lo) / h)).astype(np.int64)
    k = np.clip(np.floor((pos - lo) * (1.0 / h)), 0, dims - 1).astype(np.int64)
    vid = k[:, 0] + dims[0] * (k[:, 1] + dims[1] * k[:, 2])
    s4 = np.clip(np.floor((pos[:, 0] - lo[0]) * (1.0 / h) * 4.0), 0, 4 * dims[0] - 1).astype(np.int64)
    return np.lexsort((np.arange(len(pos)), s4 - 4 * k[:, 0], vid)).astype(np.uint32)


def check_binning(got, want, pos, lo, hi, h):
    """GPU binning (voxel_of_cell, voxel_start, sorted_ids, occ) against the oracle's:
    voxel of every cell, voxel starts and the occupied list bit for bit; each voxel's
    segment of the storage order holds exactly the oracle's cells of that voxel; and the
    order inside it is the library's documented one (storage_order)."""
    vid, start, ids, occ = got
    wvid, wstart, wids, wocc = want
    for name, g, w in (("voxel_of_cell", vid, wvid), ("voxel_start", start, wstart), ("occ", occ, wocc)):
        assert g.dtype == np.uint32 and g.shape == w.shape, name
        assert np.array_equal(g, w), name
    assert ids.dtype == np.uint32 and ids.shape == wids.shape
    V = len(start) - 1
    assert np.array_equal(vid[ids], np.repeat(np.arange(V, dtype=np.uint32), np.diff(start.astype(np.int64))))
    assert np.array_equal(ids[np.lexsort((ids, vid[ids]))], wids)
    assert np.array_equal(ids, storage_order(pos, lo, hi, h))
