"""GPU parity of the microenvironment solver and gradients (through the C ABI) against the
FP64 oracle, plus properties that hold at any size.

Bar: densities within tol * max|rho| of the oracle after the stated steps, where tol is
the smaller of 1e-10 (the FP64 bar of the method) and the rounding bound of the Thomas
solves: per step, three solves, each off by about n eps times the condition number of
its matrix, at most (b + 4r) / b; the solves are contractions, so errors add up at most
linearly over steps.  The two sides differ only in rounding: the kernels multiply by
elimination factors computed once, the oracle divides at every step.
Gradients are compared with the oracle's gradients of the GPU's own densities to a few
ulp (the same differences in another rounding order).
"""
import numpy as np
import pytest

import workloads
from gpu_helpers import require_gpu, say
from oracle import diffusion as OD
from paper_2306_11544_amd import binding as B

pytestmark = pytest.mark.gpu
EPS = np.finfo(np.float64).eps


def _tol(env, steps):
    r = np.array(env.diffusion) * env.dt / env.dx ** 2
    b = 1.0 + np.array(env.decay) * env.dt / 3.0
    kappa = float(((b + 4 * r) / b).max())
    return min(1e-10, 3.0 * max(steps, 1) * max(env.dims) * kappa * EPS)


def _run_gpu(env, steps, grads=True):
    with B.Microenv(B.microenv_params_of(env), env.density) as M:
        M.step(steps)
        if grads:
            M.compute_gradients()
        rho = M.density()
        g = M.gradients() if grads else None
    return rho, g


def _check(env, steps, case):
    say("microenv", case, env.name, "steps", steps)
    rho, g = _run_gpu(env, steps)
    p = OD.params_of(env)
    want = OD.step(p, env.density, steps)
    scale = np.abs(want).max()
    err = np.abs(rho - want).max() / scale
    tol = _tol(env, steps)
    assert err <= tol, f"{case}: density error {err:.3e} > {tol:.3e}"
    g_own = OD.gradients(p, rho)
    gs = max(np.abs(g_own).max(), scale / env.dx)
    gerr = np.abs(g - g_own).max() / gs
    assert gerr <= 64 * EPS, f"{case}: gradient error {gerr:.3e}"
    g_ora = OD.gradients(p, want)
    assert np.abs(g - g_ora).max() <= 2.0 * tol * scale / env.dx + 64 * EPS * gs
    return err


def test_paper_mesh_75_cubed_100_steps():
    require_gpu()
    env = workloads.microenv((75, 75, 75), 1, seed=6, steps=100)
    err = _check(env, 100, "75^3")
    say("75^3 density error", err)


@pytest.mark.parametrize("dims,ns,seed", [
    ((130, 7, 3), 3, 61),      # x lines longer than LDS holds: the in-place walk
    ((5, 140, 9), 2, 62),      # y lines longer than LDS holds
    ((3, 4, 200), 2, 63),      # z lines longer than LDS holds
    ((66, 65, 3), 4, 64),      # line counts that leave a ragged last block
    ((1, 1, 1), 1, 65),        # one voxel: decay only
    ((1, 70, 1), 2, 66), ((70, 1, 1), 1, 67), ((2, 1, 2), 3, 68),
    ((128, 128, 2), 1, 69),    # the longest lines staged in LDS whole
    ((112, 9, 113), 2, 76),    # the longest segmented lines (x), the shortest whole ones (z)
    ((21, 11, 19), 3, 77),     # two and three segments with a ragged last one
    ((40, 40, 40), 11, 78),    # more lines than one wave per compute unit: one lane per line
])
def test_ragged_and_multi_substrate_meshes(dims, ns, seed):
    require_gpu()
    env = workloads.microenv(dims, ns, seed=seed, steps=25)
    _check(env, 25, f"{dims}x{ns}")


def test_zero_steps_and_zero_time_step():
    require_gpu()
    env = workloads.microenv((9, 8, 7), 2, seed=70)
    rho, _ = _run_gpu(env, 0, grads=False)
    assert np.array_equal(rho, env.density)
    env.dt = 0.0   # every matrix is the identity
    rho, _ = _run_gpu(env, 3, grads=False)
    assert np.array_equal(rho, env.density)


def test_mass_conserved_without_decay_at_full_size():
    require_gpu()
    env = workloads.microenv((75, 75, 75), 2, seed=71)
    env.decay = (0.0, 0.0)
    rho, _ = _run_gpu(env, 50, grads=False)
    for s in range(2):
        m0, m1 = env.density[s].sum(), rho[s].sum()
        assert abs(m1 - m0) <= 1e-12 * m0, (s, m0, m1)


def test_cosine_mode_decays_by_the_closed_form_at_full_size():
    """Independent of the oracle: a separable cosine mode is an eigenvector of each
    solve, so after k steps it is scaled by prod_a (1 + lambda dt/3 + 4 r sin^2(pi k_a /
    (2 n_a)))^-k."""
    require_gpu()
    dims, kk, steps = (75, 75, 75), (3, 1, 2), 20
    env = workloads.microenv(dims, 1, seed=72)
    env.dt = 0.05
    nx, ny, nz = dims
    m = (np.cos(np.pi * kk[2] * (np.arange(nz) + 0.5) / nz)[:, None, None]
         * np.cos(np.pi * kk[1] * (np.arange(ny) + 0.5) / ny)[None, :, None]
         * np.cos(np.pi * kk[0] * (np.arange(nx) + 0.5) / nx)[None, None, :])
    env.density = m[None].copy()
    rho, _ = _run_gpu(env, steps, grads=False)
    r = env.diffusion[0] * env.dt / env.dx ** 2
    f = 1.0
    for a in range(3):
        f /= 1.0 + env.decay[0] * env.dt / 3.0 + 4.0 * r * np.sin(np.pi * kk[a] / (2.0 * dims[a])) ** 2
    np.testing.assert_allclose(rho[0], m * f ** steps, rtol=0, atol=1e-13)


def test_gradient_of_a_linear_field_is_exact():
    require_gpu()
    dims = (40, 33, 27)
    env = workloads.microenv(dims, 1, seed=73)
    dx = env.dx
    nx, ny, nz = dims
    z, y, x = np.meshgrid((np.arange(nz) + 0.5) * dx, (np.arange(ny) + 0.5) * dx,
                          (np.arange(nx) + 0.5) * dx, indexing="ij")
    env.density = (5.0 + 0.5 * x - 0.25 * y + 2.0 * z)[None]
    _, g = _run_gpu(env, 0)
    for a, b in enumerate((0.5, -0.25, 2.0)):
        np.testing.assert_allclose(g[0, a], b, rtol=0, atol=1e-12)


def test_graph_steps_equal_direct_launches_bitwise():
    require_gpu()
    env = workloads.microenv((33, 21, 17), 2, seed=74)
    prm = B.microenv_params_of(env)
    with B.Microenv(prm, env.density) as M:
        M.step(7)
        M.compute_gradients()
        a, ga = M.density(), M.gradients()
    with B.Microenv(prm, env.density) as M:
        ms = M.profile(7)          # direct launches, then the gradients
        b, gb = M.density(), M.gradients()
    assert np.array_equal(a, b) and np.array_equal(ga, gb)
    assert all(t > 0 for t in ms)


def test_write_density_and_size_errors():
    require_gpu()
    env = workloads.microenv((6, 5, 4), 1, seed=75)
    with B.Microenv(B.microenv_params_of(env), env.density) as M:
        new = env.density * 2.0
        M.set_density(new)
        assert np.array_equal(M.density(), new)
        with pytest.raises(B.MechError) as e:
            B._ck(B.lib().read_density(M.h, B._d(np.zeros(10)), 10))
        assert e.value.code == B.MECH_E_INVALID
        bad = new.copy()
        bad[0, 1, 2, 3] = np.nan
        with pytest.raises(B.MechError) as e:
            M.set_density(bad)
        assert e.value.code == B.MECH_E_INVALID
        d, g = M.device_arrays()
        assert d and g and M.stream
