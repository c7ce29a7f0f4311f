"""CPU oracle for the agent-mechanics step -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may import this
package.  The product path (the HIP library and its Python binding) never imports,
links or calls it, and the two share no code: the only thing both sides see is the
seeded inputs built by the `workloads` package.

The arithmetic lives in `mech_oracle.c` (plain C, FP64, -ffp-contract=off), which
states what it computes.  This module builds it with gcc and wraps it with ctypes.

Parity status of each function (what pins it is listed in tests/test_oracle_*.py):
  bin                pinned: numpy floor + lexsort, hand-built cases
  velocity_allpairs  pinned: two-cell closed forms, lattices, Newton's third law
  velocity_voxel     pinned: equals all-pairs (pair set exactly, sums to 1e-13)
  run / integrate    pinned: two-cell closed-form trajectories, exact AB2 recurrence
                     in 50-digit arithmetic, reflecting-wall special cases
  FP32 variants      pinned: the float in-range decision equals numpy's per-operation
                     float32 evaluation of the written expression on pairs within a
                     few ulps of their cutoff; decisions equal FP64 on well-separated
                     pairs; the Kahan sum within the textbook compensated-summation
                     bound of math.fsum
  velocity_sampled   pinned: equals velocity_voxel on the sampled cells
  splitmix64         pinned: the generator's published reference outputs (tests/golden)
  uniform / divide / pinned: uniformity, selection by the draws, ranks and ids, parent and
  run_growing        daughter at distance r around the parent's position (no-force
                     cases), capacity limit, walls, and p_div = 0 equal to run
  die / death_draw   pinned: survivors are exactly the cells whose draw (recomputed from
                     splitmix64 in the test) is at or above p_death, in id order with
                     their state unchanged; p_death = 0 and 1; the death and division
                     streams differ
Every function is pinned; none is "parity unpinned".  The absolute many-cell
trajectories rest on the pins above plus the comparison with the GPU path.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mech_oracle.c")
# Another build of the oracle can be loaded instead by naming it in MECH_ORACLE_LIB: the
# test that plants mistakes in copies of mech_oracle.c runs the pins against them.
_LIB = os.environ.get("MECH_ORACLE_LIB") or os.path.join(_HERE, "libmech_oracle.so")

FP64, FP32, FP32_KAHAN = 0, 1, 2


class OracleParams(C.Structure):
    _fields_ = [("lo", C.c_double * 3), ("hi", C.c_double * 3), ("h", C.c_double),
                ("dt", C.c_double), ("c_rep", C.c_double), ("alpha", C.c_double),
                ("n_types", C.c_int32), ("pad_", C.c_int32), ("c_adh", C.c_double * 64)]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (OpenMP over cells; no fast-math, no contraction),
    and the microenvironment oracle (oracle.diffusion) beside it."""
    from . import diffusion
    diffusion.build(force)
    if os.environ.get("MECH_ORACLE_LIB"):
        return _LIB
    if force or not os.path.exists(_LIB):
        compile_to(_SRC, _LIB)
    return _LIB


def compile_to(src: str, out: str) -> None:
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
           "-fno-fast-math", "-Wall", "-Wextra", "-Wno-unused-parameter", src, "-o",
           out + ".tmp", "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = C.CDLL(_LIB)
        P = C.POINTER
        dp, up, ip, lp = P(C.c_double), P(C.c_uint32), P(C.c_int32), P(C.c_int64)
        L.oracle_grid_dims.argtypes = [P(OracleParams), ip]
        L.oracle_bin.argtypes = [P(OracleParams), C.c_int64, dp, up, up, up, up, lp]
        L.oracle_velocity_allpairs.argtypes = [P(OracleParams), C.c_int64, dp, dp, ip,
                                               C.c_int32, dp, lp]
        L.oracle_velocity_voxel.argtypes = [P(OracleParams), C.c_int64, dp, dp, ip, C.c_int32,
                                            dp, lp, lp]
        L.oracle_integrate.argtypes = [P(OracleParams), C.c_int64, dp, dp, dp, C.c_int32]
        L.oracle_run.argtypes = [P(OracleParams), C.c_int64, dp, dp, ip, dp, C.c_int64,
                                 C.c_int32, C.c_int32, C.c_int32, lp, lp, lp]
        L.oracle_velocity_sampled.argtypes = [P(OracleParams), C.c_int64, dp, dp, ip,
                                              C.c_int32, C.c_int64, lp, dp, lp]
        L.oracle_set_threads.argtypes = [C.c_int32]
        L.oracle_splitmix64.argtypes = [C.c_uint64]
        L.oracle_splitmix64.restype = C.c_uint64
        L.oracle_uniform.argtypes = [C.c_uint64, C.c_uint64, C.c_uint64, C.c_uint64]
        L.oracle_uniform.restype = C.c_double
        L.oracle_divide.argtypes = [P(OracleParams), C.c_int64, C.c_int64, dp, dp, ip, dp,
                                    C.c_uint64, C.c_int64, C.c_double, lp]
        L.oracle_divide.restype = C.c_int32
        L.oracle_die.argtypes = [C.c_int64, dp, dp, ip, dp, C.c_uint64, C.c_int64, C.c_double, lp]
        L.oracle_die.restype = C.c_int32
        L.oracle_sum_f32.argtypes = [P(C.c_float), C.c_int64, C.c_int32]
        L.oracle_sum_f32.restype = C.c_float
        for f in ("oracle_grid_dims", "oracle_bin", "oracle_velocity_allpairs",
                  "oracle_velocity_voxel", "oracle_integrate", "oracle_run",
                  "oracle_velocity_sampled", "oracle_set_threads"):
            getattr(L, f).restype = C.c_int32
        _lib = L
    return _lib


def params(lo, hi, h=30.0, dt=0.1, c_rep=10.0, alpha=1.25, c_adh=((0.4,),)) -> OracleParams:
    p = OracleParams()
    for a in range(3):
        p.lo[a] = float(lo[a])
        p.hi[a] = float(hi[a])
    p.h, p.dt, p.c_rep, p.alpha = float(h), float(dt), float(c_rep), float(alpha)
    c = np.asarray(c_adh, dtype=np.float64)
    p.n_types = int(c.shape[0])
    for k, val in enumerate(c.reshape(-1)):
        p.c_adh[k] = float(val)
    return p


def params_of(pop) -> OracleParams:
    return params(pop.lo, pop.hi, pop.voxel, pop.dt, pop.c_rep, pop.alpha, pop.c_adh)


def _d(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _u(a):
    return a.ctypes.data_as(C.POINTER(C.c_uint32))


def _i(a):
    return a.ctypes.data_as(C.POINTER(C.c_int32))


def _l(a):
    return a.ctypes.data_as(C.POINTER(C.c_int64))


def _check(rc, what):
    if rc != 0:
        raise RuntimeError(f"oracle {what} failed with code {rc}")


def set_threads(t: int = 0) -> int:
    """Set the OpenMP thread count (0 keeps it); returns the count in effect."""
    return int(lib().oracle_set_threads(int(t)))


def sum_f32(x, kahan=True) -> float:
    """The FP32 velocity's accumulator applied to a plain sequence of floats."""
    x = np.ascontiguousarray(x, dtype=np.float32)
    return float(lib().oracle_sum_f32(x.ctypes.data_as(C.POINTER(C.c_float)), x.size,
                                      int(kahan)))


def grid_dims(p: OracleParams):
    d = np.zeros(3, dtype=np.int32)
    _check(lib().oracle_grid_dims(C.byref(p), _i(d)), "grid_dims")
    return tuple(int(x) for x in d)


def bin(p: OracleParams, pos):
    """Returns vid[n], voxel_start[V+1], sorted_ids[n], occ[M] (all uint32)."""
    pos = np.ascontiguousarray(pos, dtype=np.float64)
    n = pos.shape[0]
    nx, ny, nz = grid_dims(p)
    V = nx * ny * nz
    vid = np.zeros(max(n, 1), np.uint32)
    start = np.zeros(V + 1, np.uint32)
    ids = np.zeros(max(n, 1), np.uint32)
    occ = np.zeros(max(V, 1), np.uint32)
    m = np.zeros(1, np.int64)
    _check(lib().oracle_bin(C.byref(p), n, _d(pos), _u(vid), _u(start), _u(ids), _u(occ),
                            _l(m)), "bin")
    return vid[:n], start, ids[:n], occ[:int(m[0])]


def _types(t, n):
    if t is None:
        return np.zeros(max(n, 1), np.int32)
    return np.ascontiguousarray(t, dtype=np.int32)


def velocity_allpairs(p, pos, radius, types=None, precision=FP64):
    pos = np.ascontiguousarray(pos, dtype=np.float64)
    radius = np.ascontiguousarray(radius, dtype=np.float64)
    n = pos.shape[0]
    vel = np.zeros((max(n, 1), 3), np.float64)
    inter = np.zeros(1, np.int64)
    _check(lib().oracle_velocity_allpairs(C.byref(p), n, _d(pos), _d(radius),
                                          _i(_types(types, n)), precision, _d(vel),
                                          _l(inter)), "velocity_allpairs")
    return vel[:n], int(inter[0])


def velocity_voxel(p, pos, radius, types=None, precision=FP64):
    """Returns (vel[n,3] in id order, interactions, candidates)."""
    pos = np.ascontiguousarray(pos, dtype=np.float64)
    radius = np.ascontiguousarray(radius, dtype=np.float64)
    n = pos.shape[0]
    vel = np.zeros((max(n, 1), 3), np.float64)
    inter = np.zeros(1, np.int64)
    cand = np.zeros(1, np.int64)
    _check(lib().oracle_velocity_voxel(C.byref(p), n, _d(pos), _d(radius),
                                       _i(_types(types, n)), precision, _d(vel), _l(inter),
                                       _l(cand)), "velocity_voxel")
    return vel[:n], int(inter[0]), int(cand[0])


def velocity_sampled(p, pos, radius, types, sample_ids, precision=FP64):
    pos = np.ascontiguousarray(pos, dtype=np.float64)
    radius = np.ascontiguousarray(radius, dtype=np.float64)
    n = pos.shape[0]
    sid = np.ascontiguousarray(sample_ids, dtype=np.int64)
    vel = np.zeros((max(len(sid), 1), 3), np.float64)
    inter = np.zeros(1, np.int64)
    _check(lib().oracle_velocity_sampled(C.byref(p), n, _d(pos), _d(radius),
                                         _i(_types(types, n)), precision, len(sid), _l(sid),
                                         _d(vel), _l(inter)), "velocity_sampled")
    return vel[:len(sid)], int(inter[0])


def integrate(p, pos, vel, vprev, euler_start=False):
    """In place: pos, vprev (both (n,3) float64 C-contiguous)."""
    assert pos.flags.c_contiguous and vprev.flags.c_contiguous
    vel = np.ascontiguousarray(vel, dtype=np.float64)
    _check(lib().oracle_integrate(C.byref(p), pos.shape[0], _d(pos), _d(vel), _d(vprev),
                                  int(euler_start)), "integrate")


def run(p, pos, radius, types=None, vprev=None, steps=1, precision=FP64, euler_first=False,
        allpairs=False, per_step=False):
    """Advance copies of pos/vprev by `steps` steps.

    Returns dict(pos, vprev, interactions, candidates[, per_step_interactions])."""
    pos = np.array(pos, dtype=np.float64, order="C", copy=True)
    radius = np.ascontiguousarray(radius, dtype=np.float64)
    n = pos.shape[0]
    vp = (np.zeros((n, 3), np.float64) if vprev is None
          else np.array(vprev, dtype=np.float64, order="C", copy=True))
    if n == 0:
        return dict(pos=pos, vprev=vp, interactions=0, candidates=0,
                    per_step_interactions=np.zeros(steps, np.int64))
    inter = np.zeros(1, np.int64)
    cand = np.zeros(1, np.int64)
    ps = np.zeros(max(steps, 1), np.int64)
    _check(lib().oracle_run(C.byref(p), n, _d(pos), _d(radius), _i(_types(types, n)), _d(vp),
                            int(steps), int(precision), int(euler_first), int(allpairs),
                            _l(ps), _l(inter), _l(cand)), "run")
    out = dict(pos=pos, vprev=vp, interactions=int(inter[0]), candidates=int(cand[0]))
    if per_step:
        out["per_step_interactions"] = ps[:steps]
    return out


def run_pop(pop, steps=None, precision=FP64, euler_first=False, per_step=False):
    return run(params_of(pop), pop.pos, pop.radius, pop.type, None,
               pop.steps if steps is None else steps, precision, euler_first, False, per_step)


def splitmix64(state: int) -> int:
    """The SplitMix64 output function applied to one state."""
    return int(lib().oracle_splitmix64(C.c_uint64(state & ((1 << 64) - 1))))


def uniform(seed: int, cell_id: int, t: int, k: int) -> float:
    """The counter-based uniform draw of division (see oracle_divide in mech_oracle.c)."""
    return float(lib().oracle_uniform(seed, cell_id, t, k))


def death_draw(seed: int, cell_id: int, t: int) -> float:
    """The death draw of cell `cell_id` after step t (see oracle_die in mech_oracle.c)."""
    return uniform(seed ^ (1 << 63), cell_id, t, 0)


def run_growing(p: OracleParams, pos, radius, type_=None, steps: int = 1, precision: int = FP64,
                capacity: int = 0, p_div: float = 0.0, seed: int = 0, euler_first: bool = False,
                p_death: float = 0.0):
    """Steps of the method, each followed by division and then death (arrays in id
    order).  Returns dict(pos, vprev, radius, type, n, per_step_n, interactions)."""
    pos = np.ascontiguousarray(pos, dtype=np.float64).reshape(-1, 3)
    n = pos.shape[0]
    cap = max(capacity, n)
    P = np.zeros((cap, 3)); P[:n] = pos
    Rr = np.zeros(cap); Rr[:n] = radius
    T = np.zeros(cap, np.int32)
    if type_ is not None:
        T[:n] = type_
    VP = np.zeros((cap, 3))
    per_n, inter = [], 0
    L = lib()
    for t in range(steps):
        v, it, _ = velocity_voxel(p, P[:n], Rr[:n], T[:n], precision)
        inter += it
        x = np.ascontiguousarray(P[:n]); vp = np.ascontiguousarray(VP[:n])
        v = np.ascontiguousarray(v)
        _check(L.oracle_integrate(C.byref(p), n, _d(x), _d(v), _d(vp),
                                  int(euler_first and t == 0)), "integrate")
        P[:n] = x; VP[:n] = vp
        if p_div > 0.0:
            n_out = C.c_int64(0)
            _check(L.oracle_divide(C.byref(p), n, cap, _d(P), _d(Rr), _i(T), _d(VP), seed, t,
                                   float(p_div), C.byref(n_out)), "divide")
            n = int(n_out.value)
        if p_death > 0.0:
            n_out = C.c_int64(0)
            _check(L.oracle_die(n, _d(P), _d(Rr), _i(T), _d(VP), seed, t, float(p_death),
                                C.byref(n_out)), "die")
            n = int(n_out.value)
        per_n.append(n)
    return dict(pos=P[:n].copy(), vprev=VP[:n].copy(), radius=Rr[:n].copy(), type=T[:n].copy(),
                n=n, per_step_n=per_n, interactions=inter)
