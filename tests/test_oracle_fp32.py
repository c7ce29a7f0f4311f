"""Pins the FP32 variant's in-range decision to the written expression in float arithmetic.

The float decision of a pair is 0 < d2 < R_A^2 with every operation rounded to float on
its own: dx = x_i - x_j (per axis), d2 = (dx*dx + dy*dy) + dz*dz, R = r_i + r_j,
R_A = fl(alpha) * R.  numpy's float32 arithmetic rounds each elementwise operation
correctly and never fuses two of them, so it evaluates exactly that expression.  Pairs
are placed within a few float ulps of their adhesion cutoff, where a fused or
reordered d2, a dropped term or a different R_A changes some decisions; the oracle's
float pair count must equal numpy's on every one of them."""
import numpy as np
import pytest


def near_cutoff_pairs(n, seed):
    """n pairs whose exact float distance sits within a few ulps of R_A; coordinates and
    radii are floats, so the oracle's rounding of its double inputs to float is exact."""
    rng = np.random.default_rng(seed)
    r = rng.uniform(6.0, 11.0, (n, 2)).astype(np.float32)
    R = r[:, 0] + r[:, 1]
    RA = np.float32(1.25) * R
    u = rng.normal(size=(n, 3))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    d = RA.astype(np.float64) * (1.0 + rng.integers(-6, 7, n) * 2.0 ** -24)
    xi = rng.uniform(-500, 500, (n, 3)).astype(np.float32)
    xj = (xi.astype(np.float64) + u * d[:, None]).astype(np.float32)
    return xi, xj, r


def numpy_decision(xi, xj, r):
    f = np.float32
    dx = (xi[:, 0] - xj[:, 0]).astype(f)
    dy = (xi[:, 1] - xj[:, 1]).astype(f)
    dz = (xi[:, 2] - xj[:, 2]).astype(f)
    d2 = (dx * dx + dy * dy) + dz * dz
    R = r[:, 0] + r[:, 1]
    RA = f(1.25) * R
    assert d2.dtype == f and RA.dtype == f
    return (d2 > f(0)) & (d2 < RA * RA)


@pytest.mark.parametrize("precision", [1, 2])
def test_float_decision_is_the_written_expression(orc, precision):
    xi, xj, r = near_cutoff_pairs(3000, seed=41)
    want = numpy_decision(xi, xj, r)
    # both outcomes occur, so a changed expression cannot pass by always agreeing
    assert 300 < want.sum() < 2700
    p = orc.params((-1000.0,) * 3, (1000.0,) * 3, h=30.0)
    got = np.empty(len(want), bool)
    for k in range(len(want)):
        pos = np.stack([xi[k], xj[k]]).astype(np.float64)
        _, inter = orc.velocity_allpairs(p, pos, r[k].astype(np.float64), None, precision)
        assert inter in (0, 2)        # the decision is symmetric in i and j
        got[k] = inter == 2
    assert np.array_equal(got, want), int((got != want).sum())


def test_double_decision_is_the_written_expression(orc):
    """The FP64 decision on the same pairs, against numpy's float64 evaluation."""
    xi, xj, r = near_cutoff_pairs(2000, seed=42)
    a, b, rr = xi.astype(np.float64), xj.astype(np.float64), r.astype(np.float64)
    dx, dy, dz = (a - b).T
    d2 = (dx * dx + dy * dy) + dz * dz
    RA = 1.25 * (rr[:, 0] + rr[:, 1])
    want = (d2 > 0) & (d2 < RA * RA)
    p = orc.params((-1000.0,) * 3, (1000.0,) * 3, h=30.0)
    got = np.array([orc.velocity_allpairs(p, np.stack([a[k], b[k]]), rr[k])[1] == 2
                    for k in range(len(want))])
    assert np.array_equal(got, want)
