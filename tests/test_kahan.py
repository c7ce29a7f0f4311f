"""Pins the FP32 variant's compensated accumulator against math.fsum.

Kahan summation of n floats satisfies |S_kahan - S| <= (2 eps + O(n eps^2)) sum |x_i|
(Higham, Accuracy and Stability of Numerical Algorithms, Section 4.3), with eps = 2^-24
for float.  The plain float sum only meets the weaker (n - 1) eps sum |x_i| bound and
fails the compensated one on these sequences.
"""
import math

import numpy as np
import pytest

EPS = 2.0 ** -24


def sequences():
    rng = np.random.default_rng(17)
    yield "one_plus_tiny", np.concatenate([[1.0], np.full(20000, 1e-8)]).astype(np.float32)
    yield "tenths", np.full(10000, 0.1, dtype=np.float32)
    x = rng.normal(0, 1, 5000).astype(np.float32)
    yield "cancelling", np.concatenate([x, -x[::-1] * np.float32(1.0000001)]).astype(np.float32)
    yield "mixed_scale", (rng.standard_normal(4096) * 10.0 ** rng.integers(-6, 3, 4096)).astype(np.float32)
    yield "forces_like", (rng.standard_normal(60) * 5).astype(np.float32)


SEQ = list(sequences())


def exact(x):
    return math.fsum(float(v) for v in x)


@pytest.mark.parametrize("name,x", SEQ, ids=[s[0] for s in SEQ])
def test_kahan_bound(orc, name, x):
    s = orc.sum_f32(x, kahan=True)
    n = len(x)
    bound = (2 * EPS + 2 * n * EPS * EPS) * float(np.abs(x.astype(np.float64)).sum())
    assert abs(s - exact(x)) <= bound


def test_plain_sum_fails_the_compensated_bound(orc):
    fails = 0
    for name, x in SEQ:
        s = orc.sum_f32(x, kahan=False)
        n = len(x)
        bound = (2 * EPS + 2 * n * EPS * EPS) * float(np.abs(x.astype(np.float64)).sum())
        fails += abs(s - exact(x)) > bound
        # but it does meet the classical recursive-summation bound
        assert abs(s - exact(x)) <= (n - 1) * EPS * float(np.abs(x.astype(np.float64)).sum()) * 1.01 + 1e-30
    assert fails >= 2
