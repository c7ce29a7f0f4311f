"""CPU oracle for the microenvironment solver and the gradients -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may import this
module.  The arithmetic lives in `diffusion_oracle.c` (plain C, FP64, -ffp-contract=off),
which states what it computes: the locally one-dimensional implicit steps of the
diffusion-decay equation with no-flux walls (a Thomas solve per mesh line, x then y then
z) and the central-difference gradients of the substrate densities.  This module builds
it with gcc and wraps it with ctypes.

Parity status (what pins it is in tests/test_oracle_diffusion.py):
  step / sweep  pinned: a uniform field decays by exactly (1 + lambda dt / 3)^-3 per step;
                separable cosine modes are eigenvectors of the discrete operator and decay
                by the closed-form factor of each axis; mass is conserved at zero decay;
                each sweep equals a dense linear solve (numpy) of the assembled system;
                small time steps converge to the continuous mode decay
  gradients     pinned: exact on linear fields (faces included), exact on quadratic
                fields inside, the one-sided face values of a quadratic field
Every function is pinned; none is "parity unpinned".
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "diffusion_oracle.c")
# another build can be loaded instead (the planted-mistake test runs the pins on copies)
_LIB = os.environ.get("DIFF_ORACLE_LIB") or os.path.join(_HERE, "libdiffusion_oracle.so")

MAX_SUBSTRATES = 16


class DiffOracleParams(C.Structure):
    _fields_ = [("dims", C.c_int32 * 3), ("n_substrates", C.c_int32), ("dx", C.c_double),
                ("dt", C.c_double), ("diffusion", C.c_double * MAX_SUBSTRATES),
                ("decay", C.c_double * MAX_SUBSTRATES)]


def compile_to(src: str, out: str) -> None:
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
           "-fno-fast-math", "-Wall", "-Wextra", src, "-o", out + ".tmp", "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)


def build(force: bool = True) -> str:
    if os.environ.get("DIFF_ORACLE_LIB"):
        return _LIB
    if force or not os.path.exists(_LIB):
        compile_to(_SRC, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = C.CDLL(_LIB)
        P = C.POINTER
        dp = P(C.c_double)
        L.oracle_diffusion_step.argtypes = [P(DiffOracleParams), dp, C.c_int64]
        L.oracle_diffusion_sweep.argtypes = [P(DiffOracleParams), dp, C.c_int32]
        L.oracle_gradients.argtypes = [P(DiffOracleParams), dp, dp]
        for f in ("oracle_diffusion_step", "oracle_diffusion_sweep", "oracle_gradients"):
            getattr(L, f).restype = C.c_int32
        _lib = L
    return _lib


def params(dims, dx=20.0, dt=0.01, diffusion=(1e5,), decay=(0.1,)) -> DiffOracleParams:
    p = DiffOracleParams()
    for a in range(3):
        p.dims[a] = int(dims[a])
    D = np.atleast_1d(np.asarray(diffusion, dtype=np.float64))
    lam = np.atleast_1d(np.asarray(decay, dtype=np.float64))
    assert D.shape == lam.shape and 1 <= D.size <= MAX_SUBSTRATES
    p.n_substrates = int(D.size)
    p.dx, p.dt = float(dx), float(dt)
    for s in range(D.size):
        p.diffusion[s] = float(D[s])
        p.decay[s] = float(lam[s])
    return p


def params_of(env) -> DiffOracleParams:
    """From a workloads.Microenv description."""
    return params(env.dims, env.dx, env.dt, env.diffusion, env.decay)


def _d(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _field(p: DiffOracleParams, rho):
    nx, ny, nz = (int(p.dims[a]) for a in range(3))
    rho = np.array(rho, dtype=np.float64, order="C", copy=True)
    return rho.reshape(int(p.n_substrates), nz, ny, nx)


def step(p: DiffOracleParams, rho, steps: int = 1):
    """`steps` solver steps on a copy of rho[s][z][y][x]; returns the new densities."""
    u = _field(p, rho)
    rc = lib().oracle_diffusion_step(C.byref(p), _d(u), int(steps))
    if rc != 0:
        raise RuntimeError(f"oracle diffusion step failed with code {rc}")
    return u


def sweep(p: DiffOracleParams, rho, axis: int):
    """One implicit one-dimensional solve along `axis` (0 x, 1 y, 2 z) on a copy."""
    u = _field(p, rho)
    rc = lib().oracle_diffusion_sweep(C.byref(p), _d(u), int(axis))
    if rc != 0:
        raise RuntimeError(f"oracle diffusion sweep failed with code {rc}")
    return u


def gradients(p: DiffOracleParams, rho):
    """grad[s][axis][z][y][x] of rho[s][z][y][x]."""
    u = _field(p, rho)
    g = np.zeros((u.shape[0], 3) + u.shape[1:], np.float64)
    rc = lib().oracle_gradients(C.byref(p), _d(u), _d(g))
    if rc != 0:
        raise RuntimeError(f"oracle gradients failed with code {rc}")
    return g
