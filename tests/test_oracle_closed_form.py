"""Pins the oracle's force law and Adams-Bashforth update against two-cell closed forms.

Two equal cells (radius r, R = 2r, R_A = alpha*R) at separation s move symmetrically
along their axis, so s obeys ds/dt = g(s) = 2 w(s) with
    w(s) = c_rep (1 - s/R)^2 [s < R] - c_adh (1 - s/R_A)^2 [s < R_A].
For s < R, g is a quadratic with roots s* (stable) and s2, and the ODE integrates in
closed form by partial fractions; in the adhesion-only band R <= s < R_A, and for pure
repulsion, the reciprocal of the reduced gap is linear in time.  These solutions are
independent of the oracle's code, so a dropped term, a wrong sign, a wrong coefficient
or a wrong adhesion-matrix index fails one of the tests below.  The discrete
Adams-Bashforth recurrence is also evaluated exactly in 50-digit arithmetic.
"""
import math

import mpmath as mp
import numpy as np
import pytest

R_CELL = 8.4
BIG = (-60.0, -60.0, -60.0), (60.0, 60.0, 60.0)   # walls far from the pair


def _two_cell_sep(orc, s0, steps, dt, c_adh=0.4, types=(0, 0), euler=False,
                  direction=(1.0, 2.0, 2.0), matrix=None, radii=(R_CELL, R_CELL)):
    u = np.asarray(direction, float)
    u /= np.linalg.norm(u)
    pos = np.array([-0.5 * s0 * u, 0.5 * s0 * u])
    cm = matrix if matrix is not None else [[c_adh]]
    p = orc.params(*BIG, h=30.0, dt=dt, c_rep=10.0, alpha=1.25, c_adh=cm)
    out = orc.run(p, pos, np.array(radii), np.array(types, np.int32), steps=steps,
                  euler_first=euler)
    d = out["pos"][1] - out["pos"][0]
    return float(np.linalg.norm(d)), d


def _closed_form_s(s0, t, c_rep=10.0, c_adh=0.4, R=2 * R_CELL, alpha=1.25):
    """s(t) for s < R throughout (partial fractions of g = K (s - s*)(s - s2))."""
    mp.mp.dps = 40
    RA = alpha * R
    rho = mp.sqrt(mp.mpf(c_adh) / c_rep)
    K = 2 * (mp.mpf(c_rep) / R ** 2 - mp.mpf(c_adh) / RA ** 2)
    s_star = R * (1 - rho) / (1 - rho / alpha)
    s_two = R * (1 + rho) / (1 + rho / alpha)
    q0 = (s0 - s_star) / (s0 - s_two)
    q = q0 * mp.e ** (K * (s_star - s_two) * t)
    return float((s_star - s_two * q) / (1 - q)), float(s_star)


def test_equilibrium_separation_value():
    # With c_rep = 10, c_adh = 0.4, r = 8.4: sqrt(c_adh/c_rep) = 0.2 and
    # s* = 16.8 * 0.8 / (1 - 0.2/1.25) = 16 exactly.
    _, s_star = _closed_form_s(12.0, 0.0)
    assert abs(s_star - 16.0) < 1e-12


def test_pure_repulsion_closed_form(orc):
    # u = 1 - s/R obeys du/dt = -(2 c_rep / R) u^2  =>  u(t) = u0 / (1 + 2 c_rep u0 t / R)
    R = 2 * R_CELL
    u0 = 1 - 12.0 / R
    u10 = u0 / (1 + 2 * 10.0 * u0 * 10.0 / R)
    exact = R * (1 - u10)
    assert abs(exact - 15.70943) < 1e-5
    errs = []
    for dt in (0.1, 0.05, 0.025):
        s, _ = _two_cell_sep(orc, 12.0, int(round(10.0 / dt)), dt, c_adh=0.0)
        errs.append(s - exact)
    assert abs(errs[0]) < 1e-2
    # zero-history start: globally first order (error halves with dt)
    assert 1.8 < errs[0] / errs[1] < 2.2 and 1.8 < errs[1] / errs[2] < 2.2


@pytest.mark.parametrize("euler,order", [(False, 2.0), (True, 4.0)])
def test_repulsion_adhesion_closed_form(orc, euler, order):
    exact, _ = _closed_form_s(12.0, 10.0)
    assert abs(exact - 15.4450846) < 1e-6
    errs = []
    for dt in (0.1, 0.05, 0.025):
        s, d = _two_cell_sep(orc, 12.0, int(round(10.0 / dt)), dt, euler=euler)
        errs.append(s - exact)
        # the pair stays on its axis
        u = np.array([1.0, 2.0, 2.0]) / 3.0
        assert np.linalg.norm(np.cross(d / np.linalg.norm(d), u)) < 1e-12
    assert abs(errs[0]) < 5e-3
    ratio = errs[0] / errs[1]
    assert 0.85 * order < ratio < 1.15 * order, (errs, ratio)


def test_adhesion_matrix_off_diagonal(orc):
    # a type-0/type-1 pair uses C[0][1] = 0.1, whose equilibrium is
    # s* = R (1 - rho) / (1 - rho/alpha) with rho = sqrt(0.1 / 10) = 0.1
    rho = 0.1
    s_star = 2 * R_CELL * (1 - rho) / (1 - rho / 1.25)
    assert abs(s_star - 16.4347826) < 1e-6
    m = [[0.4, 0.1], [0.1, 0.4]]
    s, _ = _two_cell_sep(orc, 12.0, 3000, 0.1, types=(0, 1), matrix=m)
    assert abs(s - s_star) < 1e-6
    s_same, _ = _two_cell_sep(orc, 12.0, 3000, 0.1, types=(1, 1), matrix=m)
    assert abs(s_same - 16.0) < 1e-6


def test_adhesion_only_band(orc):
    # R <= s < R_A: w = 1 - s/R_A obeys dw/dt = (2 c_adh / R_A) w^2
    R = 2 * R_CELL
    RA = 1.25 * R
    s0, t = 20.0, 10.0
    w0 = 1 - s0 / RA
    w = 1 / (1 / w0 - 2 * 0.4 * t / RA)
    exact = RA * (1 - w)
    assert exact > R  # still inside the band at t = 10
    errs = []
    for dt in (0.1, 0.05):
        s, _ = _two_cell_sep(orc, s0, int(round(t / dt)), dt, euler=True)
        errs.append(s - exact)
    assert abs(errs[0]) < 1e-4
    assert 3.4 < errs[0] / errs[1] < 4.6


def test_unequal_radii_contact(orc):
    # unequal radii: R = r1 + r2; beyond R_A = 1.25 R nothing moves, inside it does
    r1, r2 = 6.0, 11.0
    RA = 1.25 * (r1 + r2)
    s_out, _ = _two_cell_sep(orc, RA + 1e-9, 5, 0.1, radii=(r1, r2))
    assert s_out == pytest.approx(RA + 1e-9, abs=1e-12)
    s_in, _ = _two_cell_sep(orc, RA - 1.0, 5, 0.1, radii=(r1, r2))
    assert s_in < RA - 1.0


@pytest.mark.parametrize("euler", [False, True])
@pytest.mark.parametrize("s0,c_adh", [(12.0, 0.4), (20.0, 0.4), (5.0, 0.0), (15.0, 0.1)])
def test_exact_discrete_recurrence(orc, euler, s0, c_adh):
    """The oracle's trajectory equals the AB2 recurrence evaluated in 50 digits.

    Two cells on the x axis: s_{n+1} = s_n + 2 dt (1.5 w(s_n) - 0.5 w_prev), with
    w_prev = 0 before the first step (zero history) or w(s_0) (Euler start)."""
    mp.mp.dps = 50
    R = mp.mpf(2 * R_CELL)
    RA = mp.mpf("1.25") * R
    c_rep, ca, dt = mp.mpf(10), mp.mpf(c_adh), mp.mpf("0.1")

    def w(s):
        val = mp.mpf(0)
        if s < R:
            val += c_rep * (1 - s / R) ** 2
        if s < RA:
            val -= ca * (1 - s / RA) ** 2
        return val

    steps = 100
    s = mp.mpf(s0)
    w_prev = None
    for n in range(steps):
        wn = w(s)
        wp = (wn if euler else mp.mpf(0)) if w_prev is None else w_prev
        s = s + 2 * dt * (mp.mpf("1.5") * wn - mp.mpf("0.5") * wp)
        w_prev = wn
    got, _ = _two_cell_sep(orc, s0, steps, 0.1, c_adh=c_adh, euler=euler,
                           direction=(1.0, 0.0, 0.0))
    assert abs(got - float(s)) < 1e-11, (got, float(s))


def test_equilibrium_is_stationary(orc):
    s, _ = _two_cell_sep(orc, 16.0, 200, 0.1, direction=(1.0, 0.0, 0.0))
    assert abs(s - 16.0) < 1e-13
