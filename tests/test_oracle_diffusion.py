"""Pins of the microenvironment oracle (diffusion-decay solver and gradients).

Each pin is fixed by the mathematics of the discrete scheme, not by the oracle's code:
closed-form eigen decay of the discrete operator, exact conservation, a dense linear
solve by numpy of the assembled one-dimensional systems, convergence to the continuous
mode decay, and finite-difference identities on polynomial fields.
"""
import numpy as np
import pytest

from oracle import diffusion as OD


def _coords(dims, dx):
    nx, ny, nz = dims
    z, y, x = np.meshgrid((np.arange(nz) + 0.5) * dx, (np.arange(ny) + 0.5) * dx,
                          (np.arange(nx) + 0.5) * dx, indexing="ij")
    return x, y, z


def _mode(dims, k):
    """prod_a cos(pi k_a (i_a + 1/2) / n_a) on the mesh, [z][y][x]."""
    nx, ny, nz = dims
    cx = np.cos(np.pi * k[0] * (np.arange(nx) + 0.5) / nx)
    cy = np.cos(np.pi * k[1] * (np.arange(ny) + 0.5) / ny)
    cz = np.cos(np.pi * k[2] * (np.arange(nz) + 0.5) / nz)
    return cz[:, None, None] * cy[None, :, None] * cx[None, None, :]


def _mode_factor(dims, k, r, lam_dt):
    """Per-step factor of a cosine mode: each sweep divides it by
    1 + lambda dt / 3 + 4 r sin^2(pi k_a / (2 n_a)), the eigenvalue of the sweep's matrix
    for that mode (the cell-centred Neumann Laplacian's eigenvectors are these cosines)."""
    f = 1.0
    for a in range(3):
        f /= 1.0 + lam_dt / 3.0 + 4.0 * r * np.sin(np.pi * k[a] / (2.0 * dims[a])) ** 2
    return f


@pytest.mark.parametrize("steps", [1, 5])
def test_uniform_field_decays_by_the_split_factor(steps):
    dims = (7, 5, 3)
    D, lam, dt = (1e5, 500.0, 0.0), (0.1, 2.0, 0.7), 0.5
    p = OD.params(dims, dx=20.0, dt=dt, diffusion=D, decay=lam)
    rho = np.stack([np.full(dims[::-1], c) for c in (38.0, 1.5, 1e-3)])
    out = OD.step(p, rho, steps)
    for s in range(3):
        want = rho[s, 0, 0, 0] * (1.0 + lam[s] * dt / 3.0) ** (-3 * steps)
        # rounding of a Thomas solve: about n eps times the condition number of its
        # matrix, at most (b + 4r) / b; three solves per step
        b, r = 1.0 + lam[s] * dt / 3.0, D[s] * dt / 20.0 ** 2
        tol = 3 * steps * max(dims) * (b + 4.0 * r) / b * np.finfo(float).eps
        np.testing.assert_allclose(out[s], want, rtol=tol, atol=0)


@pytest.mark.parametrize("k", [(0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1), (2, 3, 1), (7, 5, 4),
                               (3, 0, 2)])
def test_cosine_modes_decay_by_the_closed_form(k):
    dims = (8, 6, 5)
    dx, dt = 20.0, 0.25
    D = (1600.0, 40.0)           # r = 1 and 0.025
    lam = (0.3, 1.7)
    p = OD.params(dims, dx=dx, dt=dt, diffusion=D, decay=lam)
    m = _mode(dims, k)
    rho = np.stack([m, 2.0 * m])
    out = OD.step(p, rho, 2)
    for s in range(2):
        f = _mode_factor(dims, k, D[s] * dt / dx ** 2, lam[s] * dt)
        np.testing.assert_allclose(out[s], rho[s] * f * f, rtol=0, atol=1e-14 * np.abs(rho[s]).max())


@pytest.mark.parametrize("dims", [(9, 4, 6), (1, 7, 3), (5, 1, 1)])
def test_mass_is_conserved_without_decay(dims):
    rng = np.random.default_rng(11)
    p = OD.params(dims, dx=20.0, dt=0.5, diffusion=(1e5, 3.0), decay=(0.0, 0.0))
    rho = rng.uniform(0.0, 10.0, (2,) + dims[::-1])
    out = OD.step(p, rho, 10)
    for s in range(2):
        assert abs(out[s].sum() - rho[s].sum()) <= 1e-13 * rho[s].sum()
    # and decay takes it down by exactly the uniform factor per step
    p2 = OD.params(dims, dx=20.0, dt=0.5, diffusion=(1e5, 3.0), decay=(0.4, 0.4))
    out2 = OD.step(p2, rho, 3)
    f = (1.0 + 0.4 * 0.5 / 3.0) ** -9
    for s in range(2):
        assert abs(out2[s].sum() - f * rho[s].sum()) <= 1e-13 * rho[s].sum()


def _line_matrix(n, r, b):
    """The one-dimensional system of a sweep, assembled from the equation: diagonal
    b + 2r inside and b + r on the two face rows (no flux), off-diagonals -r."""
    A = np.zeros((n, n))
    for i in range(n):
        A[i, i] = b + (0 if n == 1 else r if i in (0, n - 1) else 2 * r)
        if i > 0:
            A[i, i - 1] = -r
        if i < n - 1:
            A[i, i + 1] = -r
    return A


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_each_sweep_is_the_dense_solve(axis):
    dims = (6, 5, 4)
    dx, dt, D, lam = 20.0, 0.2, (4000.0, 90.0), (0.05, 3.0)
    rng = np.random.default_rng(5 + axis)
    rho = rng.uniform(-1.0, 4.0, (2,) + dims[::-1])
    p = OD.params(dims, dx=dx, dt=dt, diffusion=D, decay=lam)
    out = OD.sweep(p, rho, axis)
    for s in range(2):
        A = _line_matrix(dims[axis], D[s] * dt / dx ** 2, 1.0 + lam[s] * dt / 3.0)
        # lines along the axis: move it last ([z][y][x] has x at -1, y at -2, z at -3)
        f = np.moveaxis(rho[s], 2 - axis, -1)
        want = np.linalg.solve(A, f.reshape(-1, dims[axis]).T).T.reshape(f.shape)
        want = np.moveaxis(want, -1, 2 - axis)
        np.testing.assert_allclose(out[s], want, rtol=0, atol=1e-13 * np.abs(rho[s]).max())


def test_step_is_the_three_sweeps_in_order():
    dims = (5, 4, 3)
    p = OD.params(dims, dx=10.0, dt=0.3, diffusion=(700.0,), decay=(0.2,))
    rho = np.random.default_rng(2).uniform(0, 1, (1,) + dims[::-1])
    want = OD.sweep(p, OD.sweep(p, OD.sweep(p, rho, 0), 1), 2)
    np.testing.assert_array_equal(OD.step(p, rho, 1), want)


def test_small_steps_converge_to_the_continuous_decay():
    """The scheme approximates d rho/dt = D lap rho - lambda rho: a mode cos(kappa x) with
    kappa = pi / L decays like exp(-(D kappa^2 + lambda) t) as dx and dt shrink."""
    L, T, D, lam = 1000.0, 2.0, 2e4, 0.3
    errs = []
    for n, dt in ((25, 0.02), (50, 0.005)):
        dims = (n, 1, 1)
        dx = L / n
        p = OD.params(dims, dx=dx, dt=dt, diffusion=(D,), decay=(lam,))
        rho = _mode(dims, (1, 0, 0))[None]
        out = OD.step(p, rho, int(round(T / dt)))
        want = rho * np.exp(-(D * (np.pi / L) ** 2 + lam) * T)
        errs.append(np.abs(out - want).max() / np.abs(want).max())
    assert errs[0] < 2e-2 and errs[1] < errs[0] / 3.0, errs


def test_gradient_of_a_linear_field_is_exact_everywhere():
    dims = (6, 5, 4)
    dx = 20.0
    x, y, z = _coords(dims, dx)
    bx, by, bz = 0.25, -1.5, 3.0
    rho = np.stack([7.0 + bx * x + by * y + bz * z, -2.0 * z])
    p = OD.params(dims, dx=dx, diffusion=(1.0, 1.0), decay=(0.0, 0.0))
    g = OD.gradients(p, rho)
    for a, b in enumerate((bx, by, bz)):
        np.testing.assert_allclose(g[0, a], b, rtol=0, atol=1e-12)
    np.testing.assert_allclose(g[1, 0], 0.0, atol=1e-12)
    np.testing.assert_allclose(g[1, 1], 0.0, atol=1e-12)
    np.testing.assert_allclose(g[1, 2], -2.0, atol=1e-12)


def test_gradient_of_a_quadratic_field_central_inside_one_sided_at_faces():
    dims = (7, 6, 5)
    dx = 10.0
    x, y, z = _coords(dims, dx)
    rho = (x * x + 3.0 * y * y - z * z)[None]
    p = OD.params(dims, dx=dx, diffusion=(1.0,), decay=(0.0,))
    g = OD.gradients(p, rho)[0]
    for a, (c, coef) in enumerate(((x, 1.0), (y, 3.0), (z, -1.0))):
        want = 2.0 * coef * c                   # central difference is exact on quadratics
        # one-sided on the faces: (f(c0 + dx) - f(c0)) / dx = coef (2 c0 + dx), and
        # (f(c) - f(c - dx)) / dx = coef (2 c - dx) on the last voxel
        idx_first = [slice(None)] * 3
        idx_last = [slice(None)] * 3
        idx_first[2 - a] = 0
        idx_last[2 - a] = -1
        want[tuple(idx_first)] = coef * (2.0 * c[tuple(idx_first)] + dx)
        want[tuple(idx_last)] = coef * (2.0 * c[tuple(idx_last)] - dx)
        np.testing.assert_allclose(g[a], want, rtol=0, atol=1e-11)


def test_gradient_along_a_single_voxel_axis_is_zero():
    dims = (4, 1, 3)
    rho = np.random.default_rng(0).uniform(0, 1, (1, 3, 1, 4))
    g = OD.gradients(OD.params(dims, dx=5.0, diffusion=(1.0,), decay=(0.0,)), rho)
    assert np.all(g[0, 1] == 0.0)


def test_invalid_parameters_are_rejected():
    with pytest.raises(RuntimeError):
        OD.step(OD.params((4, 4, 4), diffusion=(-1.0,), decay=(0.0,)), np.zeros((1, 4, 4, 4)))
    with pytest.raises(RuntimeError):
        OD.step(OD.params((4, 4, 4), dx=0.0), np.zeros((1, 4, 4, 4)))
