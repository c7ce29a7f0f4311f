"""Positions from the HIP path match the oracle after the stated step counts.

Error metric: max over cells and axes of |x_gpu - x_oracle| / S, with S the domain
half-width (positions near 0 make a per-component relative error meaningless).
Bars: 1e-10 in FP64, 1e-4 in FP32 and FP32 + Kahan (both against the FP64 oracle).
Interaction counts are integers decided in the same precision on both sides and are
compared exactly on the first step; over a trajectory only a pair within rounding of
its cutoff may differ, so later steps allow a handful of flips."""
import numpy as np
import pytest

import workloads
from gpu_helpers import assert_well_posed, disp_err, pos_err, record, require_gpu, run_gpu, say
from paper_2306_11544_amd import binding as B

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-10
FP32_TOL = 1e-4

_ORACLE_RUNS = {}


def _oracle_full(orc, name):
    """The oracle's FP64 run of a named workload for its full step count (computed once)."""
    if name not in _ORACLE_RUNS:
        _ORACLE_RUNS[name] = orc.run_pop(workloads.config(name))
    return _ORACLE_RUNS[name]


def _scaled_tumour(n, seed):
    f = (n / 1e6) ** (1 / 3)
    return workloads.tumour(n, seed=seed, core_radius=600 * f, half=1000 * f)


@pytest.mark.parametrize("name,maker,steps", [
    ("plain1k", lambda: workloads.plain(), 100),
    ("sph20k", lambda: workloads.spheroid(20000, seed=21), 200),
    ("tumour20k", lambda: _scaled_tumour(20000, 22), 100),
    ("ragged1001", lambda: workloads.spheroid(1001, seed=23), 150),
])
def test_fp64_trajectory(orc, name, maker, steps):
    require_gpu()
    pop = maker()
    assert_well_posed(orc, pop, steps)
    say("fp64", name, pop.n, steps)
    want = orc.run_pop(pop, steps=steps, per_step=True)
    got = run_gpu(pop, steps, per_step=True)
    err = pos_err(got["pos"], want["pos"], pop.half_width)
    record(f"fp64 {name} {steps} steps", err, disp_rel=disp_err(got["pos"], want["pos"], pop.pos))
    assert err <= FP64_TOL, err
    # v_prev after the last step is that step's velocity
    assert np.abs(got["vel"] - want["vprev"]).max() <= 1e-9 * max(1.0, np.abs(want["vprev"]).max())
    assert got["per_step"][0] == want["per_step_interactions"][0]
    assert np.abs(got["per_step"] - want["per_step_interactions"]).max() <= 2
    # the default kernel tests only the x slabs within reach: a subset of the 27 voxels
    assert 0 < got["candidates"] <= want["candidates"]


_FP32_CASES = [
    ("plain1k", lambda: workloads.plain(), 100),
    ("sph20k", lambda: workloads.spheroid(20000, seed=21), 200),
    ("tumour20k", lambda: _scaled_tumour(20000, 22), 100),
]


@pytest.mark.parametrize("name,maker,steps", _FP32_CASES, ids=[c[0] for c in _FP32_CASES])
def test_fp32_and_kahan_error_vs_fp64_oracle(orc, name, maker, steps):
    """The FP32 forms against the FP64 oracle on the small configurations, with the error
    of each recorded (the 1M-cell and 100k-cell cases have tests of their own)."""
    require_gpu()
    pop = maker()
    want = orc.run_pop(pop, steps=steps)
    for prec, label in ((B.MECH_FP32, "fp32"), (B.MECH_FP32_KAHAN, "fp32k")):
        got = run_gpu(pop, steps, precision=prec)
        err = pos_err(got["pos"], want["pos"], pop.half_width)
        record(f"{label} {name} {steps} steps vs fp64 oracle", err,
               disp_rel=disp_err(got["pos"], want["pos"], pop.pos))
        assert err <= FP32_TOL, (label, err)


@pytest.mark.parametrize("kernel", ["rows", "voxel"])
def test_full_neighbourhood_kernels_visit_every_candidate(orc, kernel):
    """The kernels without the slab window test every pair of the 27-voxel
    neighbourhoods: their candidate counts equal the oracle's exactly."""
    require_gpu()
    pop = _scaled_tumour(20000, 26)
    got = run_gpu(pop, 1, flags=B.FORCE_KERNELS[kernel])
    _, inter, cand = orc.velocity_voxel(orc.params_of(pop), pop.pos, pop.radius, pop.type, orc.FP64)
    assert got["interactions"] == inter
    assert got["candidates"] == cand


def test_fp64_spheroid_full_1000_steps(orc):
    """The 100k-cell two-type spheroid for its full 1,000 steps."""
    require_gpu()
    pop = workloads.config("sph100k")
    say("fp64 sph100k 1000 steps")
    got = run_gpu(pop, pop.steps)
    want = _oracle_full(orc, "sph100k")
    err = pos_err(got["pos"], want["pos"], pop.half_width)
    record("fp64 sph100k 1000 steps", err, disp_rel=disp_err(got["pos"], want["pos"], pop.pos),
           interactions=got["interactions"],
           oracle_interactions=want["interactions"])
    assert err <= FP64_TOL, err
    assert abs(got["interactions"] - want["interactions"]) <= 1e-9 * want["interactions"] + 2


@pytest.mark.parametrize("precision", [B.MECH_FP32, B.MECH_FP32_KAHAN])
def test_fp32_spheroid_full_1000_steps(orc, precision):
    require_gpu()
    pop = workloads.config("sph100k")
    say("fp32 sph100k 1000 steps", precision)
    got = run_gpu(pop, pop.steps, precision=precision)
    want = _oracle_full(orc, "sph100k")
    err = pos_err(got["pos"], want["pos"], pop.half_width)
    record(f"{'fp32k' if precision == B.MECH_FP32_KAHAN else 'fp32'} sph100k 1000 steps "
           "vs fp64 oracle", err, disp_rel=disp_err(got["pos"], want["pos"], pop.pos))
    assert err <= FP32_TOL, err


@pytest.mark.parametrize("precision", [B.MECH_FP32, B.MECH_FP32_KAHAN])
def test_fp32_first_step_decisions_exact(orc, precision):
    """Same float decisions as the oracle's float variant: equal counts on step 1,
    velocities close to the float oracle's."""
    require_gpu()
    pop = workloads.spheroid(50000, seed=24)
    say("fp32 step1", precision)
    got = run_gpu(pop, 1, precision=precision)
    want = orc.run_pop(pop, steps=1, precision=precision)
    assert got["interactions"] == want["interactions"]
    scale = np.abs(want["vprev"]).max()
    assert np.abs(got["vel"] - want["vprev"]).max() <= 2e-5 * scale


def test_kahan_compensation_is_live(orc):
    """The compensated sums are not compiled away: on a pile of cells with about 170
    neighbours each, FP32 + Kahan differs from the plain FP32 sums, and both stay as
    close to the FP64 oracle as the oracle's own float variants (the errors are
    recorded; rounding the positions to float dominates them at this size)."""
    require_gpu()
    rng = np.random.default_rng(27)
    # a dense pile: 4000 cells in a 60 um ball, deep in each other's repulsion range
    n = 4000
    d = rng.normal(size=(n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    pos = d * (60.0 * rng.uniform(0, 1, (n, 1)) ** (1 / 3))
    pop = workloads.Population(name="pile4k", pos=pos, radius=np.full(n, 8.4), type=np.zeros(n, np.int32),
                               lo=(-200.0, -200.0, -200.0), hi=(200.0, 200.0, 200.0),
                               c_adh=workloads.C_ADH_1, steps=1)
    say("kahan pile")
    plain = run_gpu(pop, 1, precision=B.MECH_FP32)["vel"]
    comp = run_gpu(pop, 1, precision=B.MECH_FP32_KAHAN)["vel"]
    exact = orc.run_pop(pop, steps=1)["vprev"]
    o_plain = orc.run_pop(pop, steps=1, precision=orc.FP32)["vprev"]
    o_comp = orc.run_pop(pop, steps=1, precision=orc.FP32_KAHAN)["vprev"]
    assert not np.array_equal(plain, comp)
    err = lambda v: float(np.abs(v - exact).max())
    assert err(comp) <= 2 * err(o_comp) + 1e-6 * np.abs(exact).max()
    assert err(plain) <= 2 * err(o_plain) + 1e-6 * np.abs(exact).max()
    record("kahan pile4k step-1 velocity max error, fp32 / fp32k / oracle fp32 / oracle fp32k",
           err(plain), fp32k=err(comp), oracle_fp32=err(o_plain), oracle_fp32k=err(o_comp))


def test_tumour1m_first_step_sampled(orc):
    """The 1M-cell tumour in FP32 + Kahan at full size: first-step velocities of sampled
    cells (each computed alone by the oracle) and the exact interaction count."""
    require_gpu()
    pop = workloads.config("tumour1m")
    say("tumour1m fp32k step 1")
    got = run_gpu(pop, 1, precision=B.MECH_FP32_KAHAN)
    rng = np.random.default_rng(25)
    ids = rng.choice(pop.n, 4000, replace=False)
    p = orc.params_of(pop)
    v32, _ = orc.velocity_sampled(p, pop.pos, pop.radius, pop.type, ids, orc.FP32_KAHAN)
    v64, _ = orc.velocity_sampled(p, pop.pos, pop.radius, pop.type, ids, orc.FP64)
    scale = np.abs(v64).max()
    record("fp32k tumour1m step-1 velocity vs fp32k oracle (rel. to max|v|)",
           np.abs(got["vel"][ids] - v32).max() / scale)
    record("fp32k tumour1m step-1 velocity vs fp64 oracle (rel. to max|v|)",
           np.abs(got["vel"][ids] - v64).max() / scale)
    assert np.abs(got["vel"][ids] - v32).max() <= 2e-5 * scale
    assert np.abs(got["vel"][ids] - v64).max() <= 1e-4 * scale
    _, inter, cand = orc.velocity_voxel(p, pop.pos, pop.radius, pop.type, orc.FP32_KAHAN)
    assert got["interactions"] == inter
    assert 0 < got["candidates"] <= cand
    # Newton's third law over the whole population
    assert np.abs(got["vel"].sum(axis=0)).max() <= 1e-5 * np.abs(got["vel"]).sum()


def test_tumour1m_full_200_steps(orc):
    """The 1M-cell tumour at full size for its stated 200 steps: the FP64 path and the
    FP32 + Kahan path against the FP64 oracle, run on the host's cores in chunks of 20
    steps (each chunk resumes from the last positions and v_prev, as the method does)."""
    require_gpu()
    pop = workloads.config("tumour1m")
    p = orc.params_of(pop)
    pos, vprev, inter = pop.pos, None, 0
    for k in range(10):
        out = orc.run(p, pos, pop.radius, pop.type, vprev, steps=20)
        pos, vprev, inter = out["pos"], out["vprev"], inter + out["interactions"]
        say("tumour1m fp64 oracle", 20 * (k + 1), "of", pop.steps, "steps")
    for precision, tol, label in ((B.MECH_FP64, FP64_TOL, "fp64"),
                                  (B.MECH_FP32_KAHAN, FP32_TOL, "fp32k")):
        got = run_gpu(pop, pop.steps, precision=precision)
        err = pos_err(got["pos"], pos, pop.half_width)
        record(f"{label} tumour1m {pop.steps} steps vs fp64 oracle", err,
               disp_rel=disp_err(got["pos"], pos, pop.pos), interactions=got["interactions"],
               oracle_interactions=inter)
        assert err <= tol, (label, err)
        if precision == B.MECH_FP64:
            assert abs(got["interactions"] - inter) <= 1e-9 * inter + 2


def test_tumour1m_full_run_properties():
    """All 200 steps at full size: state finite, inside the walls, momentum balanced."""
    require_gpu()
    pop = workloads.config("tumour1m")
    say("tumour1m fp32k 200 steps")
    got = run_gpu(pop, pop.steps, precision=B.MECH_FP32_KAHAN)
    lo, hi = np.array(pop.lo), np.array(pop.hi)
    assert np.all(got["pos"] >= lo) and np.all(got["pos"] <= hi)
    assert np.abs(got["vel"].sum(axis=0)).max() <= 1e-4 * np.abs(got["vel"]).sum()
    assert got["interactions"] > 200 * 3e7


def test_euler_start(orc):
    require_gpu()
    pop = workloads.plain()
    say("euler start")
    got = run_gpu(pop, 100, ab2_start=B.MECH_AB2_EULER_START)
    want = orc.run_pop(pop, steps=100, euler_first=True)
    err = pos_err(got["pos"], want["pos"], pop.half_width)
    record("fp64 plain1k euler start 100 steps", err, disp_rel=disp_err(got["pos"], want["pos"], pop.pos))
    assert err <= FP64_TOL
    zero = orc.run_pop(pop, steps=100)
    assert pos_err(zero["pos"], want["pos"], pop.half_width) > 1e-8  # the start matters


def test_two_cell_closed_form_on_gpu():
    """The two-cell trajectory of the GPU path against the closed-form separation."""
    require_gpu()
    import mpmath as mp
    pop = workloads.plain(2, seed=1)
    u = np.array([1.0, 2.0, 2.0]) / 3.0
    pop.pos = np.array([-6.0 * u, 6.0 * u])
    pop.radius = np.array([8.4, 8.4])
    R, RA = 16.8, 21.0
    rho = mp.sqrt(mp.mpf("0.04"))
    K = 2 * (10 / mp.mpf(R) ** 2 - mp.mpf("0.4") / mp.mpf(RA) ** 2)
    s1 = R * (1 - rho) / (1 - rho / 1.25)
    s2 = R * (1 + rho) / (1 + rho / 1.25)
    q = (12 - s1) / (12 - s2) * mp.e ** (K * (s1 - s2) * 10)
    exact = float((s1 - s2 * q) / (1 - q))
    got = run_gpu(pop, 100, ab2_start=B.MECH_AB2_EULER_START)
    s = np.linalg.norm(got["pos"][1] - got["pos"][0])
    assert abs(s - exact) < 5e-4
