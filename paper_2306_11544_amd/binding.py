"""ctypes binding of libmech.so: the C-ABI entry points under the same names.

Argument marshalling only: every step of the mechanics path runs in the HIP kernels
behind these calls.  If libmech.so has not been built this module raises on first use;
there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmech.so")

MECH_OK = 0
MECH_E_INVALID, MECH_E_VOXEL_TOO_SMALL, MECH_E_OUT_OF_DOMAIN = -1, -2, -3
MECH_E_NOMEM, MECH_E_BUDGET, MECH_E_DEVICE, MECH_E_NONFINITE, MECH_E_FULL = -4, -5, -6, -7, -8
MECH_FP64, MECH_FP32, MECH_FP32_KAHAN = 0, 1, 2
MECH_AB2_ZERO_HISTORY, MECH_AB2_EULER_START = 0, 1
MECH_FLAG_NO_GRAPH = 1
MECH_FLAG_SIMPLE_FORCE = 2
MECH_FLAG_VOXEL_FORCE = 4
MECH_FLAG_PRUNED_FORCE = 8
MECH_FORCE_KERNEL_MASK = 14
FORCE_KERNELS = {"cells": 0, "rows": MECH_FLAG_SIMPLE_FORCE, "voxel": MECH_FLAG_VOXEL_FORCE,
                 "pruned": MECH_FLAG_PRUNED_FORCE}
MECH_ABI_VERSION = 2

PRECISIONS = {"fp64": MECH_FP64, "fp32": MECH_FP32, "fp32k": MECH_FP32_KAHAN}

# every symbol include/mech.h declares
EXPORTS = ("mech_last_error", "mech_abi_version", "mech_device_count",
           "population_workspace_bytes", "create_population", "create_population_in",
           "step_mechanics", "read_state", "read_binning", "read_stats", "read_xcd_split",
           "profile_step",
           "create_population_cap", "population_set_division", "population_set_death",
           "population_size",
           "population_set_reorder", "population_get_tuning", "population_set_tuning",
           "population_info", "population_stream", "destroy_population",
           "batch_workspace_bytes", "batch_request_voxels", "create_batch", "create_batch_in",
           "batch_admit", "batch_step", "batch_poll", "batch_read", "batch_retire",
           "batch_slot_info", "batch_info", "batch_stats", "batch_profile", "batch_set_flags",
           "batch_get_tuning", "batch_set_tuning", "batch_sync", "batch_stream", "destroy_batch",
           "batch_budget_capacity", "create_batch_budget", "batch_capacity", "batch_mark_clock",
           "batch_slot_done_ms", "step_mechanics_noalloc")
MECH_NOALLOC_SCRATCH_BYTES = 64 << 20
# every symbol include/microenv.h declares
MICROENV_EXPORTS = ("create_microenvironment", "microenvironment_step", "microenvironment_gradients",
                    "read_density", "read_gradients", "write_density", "microenvironment_profile",
                    "microenvironment_device_arrays", "microenvironment_stream",
                    "destroy_microenvironment")
MECH_MAX_SUBSTRATES = 16


class MechError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"[{code}] {msg}")
        self.code = code


class MechParams(C.Structure):
    _fields_ = [("abi_version", C.c_int32), ("precision", C.c_int32), ("ab2_start", C.c_int32),
                ("flags", C.c_int32), ("domain_lo", C.c_double * 3), ("domain_hi", C.c_double * 3),
                ("voxel_size", C.c_double), ("dt", C.c_double), ("c_rep", C.c_double),
                ("rel_adh_distance", C.c_double), ("n_types", C.c_int32), ("reserved", C.c_int32),
                ("c_adh", C.c_double * 64)]


class MechMicroenvParams(C.Structure):
    _fields_ = [("abi_version", C.c_int32), ("n_substrates", C.c_int32), ("dims", C.c_int32 * 3),
                ("reserved", C.c_int32), ("voxel_size", C.c_double), ("dt", C.c_double),
                ("diffusion", C.c_double * MECH_MAX_SUBSTRATES),
                ("decay", C.c_double * MECH_MAX_SUBSTRATES)]


class MechTuning(C.Structure):
    _fields_ = [("force_kernel", C.c_int32), ("block_waves", C.c_int32), ("unroll", C.c_int32),
                ("blocks_per_cu", C.c_int32), ("list_len", C.c_int32)]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


def tuning(force_kernel=0, block_waves=1, unroll=8, blocks_per_cu=0, list_len=0) -> MechTuning:
    if isinstance(force_kernel, str):
        force_kernel = FORCE_KERNELS[force_kernel]
    return MechTuning(int(force_kernel), int(block_waves), int(unroll), int(blocks_per_cu),
                      int(list_len))


_lib = None


def lib():
    """Load libmech.so (raises if it is missing: build it with paper_2306_11544_amd.build)."""
    global _lib
    if _lib is None:
        try:
            # torch ships its own HIP runtime; loading it first makes libmech.so bind to
            # that same runtime, so torch streams and memory are valid in both
            import torch  # noqa: F401
        except ImportError:
            pass
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: run `python -m paper_2306_11544_amd.build` "
                              "(the mechanics step has no CPU fallback)")
        L = C.CDLL(LIB_PATH)
        P = C.POINTER
        vp, dp, ip, up, lp = C.c_void_p, P(C.c_double), P(C.c_int32), P(C.c_uint32), P(C.c_int64)
        sig = {
            "mech_last_error": (C.c_char_p, []),
            "mech_abi_version": (C.c_int32, []),
            "mech_device_count": (C.c_int32, []),
            "population_workspace_bytes": (C.c_int64, [P(MechParams), C.c_int64]),
            "create_population": (C.c_int, [P(MechParams), C.c_int64, dp, dp, ip, dp, vp, P(vp)]),
            "create_population_in": (C.c_int, [P(MechParams), C.c_int64, dp, dp, ip, dp, vp, vp,
                                               C.c_int64, P(vp)]),
            "step_mechanics": (C.c_int, [vp, C.c_int64]),
            "read_state": (C.c_int, [vp, dp, dp, C.c_int64]),
            "read_binning": (C.c_int, [vp, up, up, up, up, lp, lp]),
            "read_stats": (C.c_int, [vp, lp, lp, lp]),
            "read_xcd_split": (C.c_int, [vp, C.POINTER(C.c_uint32)]),
            "profile_step": (C.c_int, [vp, C.c_int64, dp]),
            "create_population_cap": (C.c_int, [P(MechParams), C.c_int64, C.c_int64, dp, dp, ip,
                                                dp, vp, P(vp)]),
            "population_set_division": (C.c_int, [vp, C.c_double, C.c_uint64]),
            "population_set_death": (C.c_int, [vp, C.c_double]),
            "population_size": (C.c_int, [vp, lp]),
            "population_set_reorder": (C.c_int, [vp, C.c_int32]),
            "population_get_tuning": (C.c_int, [vp, P(MechTuning)]),
            "population_set_tuning": (C.c_int, [vp, P(MechTuning)]),
            "population_info": (C.c_int, [vp, lp, ip]),
            "population_stream": (C.c_void_p, [vp]),
            "destroy_population": (C.c_int, [vp]),
            "batch_workspace_bytes": (C.c_int64, [P(MechParams), C.c_int64, C.c_int64, C.c_int32]),
            "batch_request_voxels": (C.c_int64, [P(MechParams), dp, dp]),
            "create_batch": (C.c_int, [P(MechParams), C.c_int64, C.c_int64, C.c_int32, vp, P(vp)]),
            "create_batch_in": (C.c_int, [P(MechParams), C.c_int64, C.c_int64, C.c_int32, vp, vp,
                                          C.c_int64, P(vp)]),
            "batch_admit": (C.c_int, [vp, dp, dp, C.c_int64, dp, dp, ip, dp, C.c_int64, ip]),
            "batch_step": (C.c_int, [vp, C.c_int64]),
            "batch_poll": (C.c_int, [vp, ip, C.c_int32, ip]),
            "batch_read": (C.c_int, [vp, C.c_int32, dp, dp, C.c_int64]),
            "batch_retire": (C.c_int, [vp, C.c_int32]),
            "batch_slot_info": (C.c_int, [vp, C.c_int32, lp, lp]),
            "batch_info": (C.c_int, [vp, lp, lp, ip, lp, lp]),
            "batch_stats": (C.c_int, [vp, lp, lp, lp]),
            "batch_profile": (C.c_int, [vp, C.c_int64, dp]),
            "batch_set_flags": (C.c_int, [vp, C.c_int32]),
            "batch_get_tuning": (C.c_int, [vp, P(MechTuning)]),
            "batch_set_tuning": (C.c_int, [vp, P(MechTuning)]),
            "batch_sync": (C.c_int, [vp]),
            "batch_stream": (C.c_void_p, [vp]),
            "destroy_batch": (C.c_int, [vp]),
            "batch_budget_capacity": (C.c_int, [P(MechParams), C.c_int64, C.c_double, C.c_int32, lp, lp]),
            "create_batch_budget": (C.c_int, [P(MechParams), C.c_int64, C.c_double, C.c_int32, vp, P(vp)]),
            "batch_capacity": (C.c_int, [vp, lp, lp, ip, lp]),
            "batch_mark_clock": (C.c_int, [vp]),
            "batch_slot_done_ms": (C.c_int, [vp, C.c_int32, dp]),
            "step_mechanics_noalloc": (C.c_int, [P(MechParams), C.c_int64, dp, dp, ip, dp, C.c_int64, vp,
                                                 dp, dp, lp]),
            "create_microenvironment": (C.c_int, [P(MechMicroenvParams), dp, vp, P(vp)]),
            "microenvironment_step": (C.c_int, [vp, C.c_int64]),
            "microenvironment_gradients": (C.c_int, [vp]),
            "read_density": (C.c_int, [vp, dp, C.c_int64]),
            "read_gradients": (C.c_int, [vp, dp, C.c_int64]),
            "write_density": (C.c_int, [vp, dp, C.c_int64]),
            "microenvironment_profile": (C.c_int, [vp, C.c_int64, dp]),
            "microenvironment_device_arrays": (C.c_int, [vp, P(vp), P(vp)]),
            "microenvironment_stream": (C.c_void_p, [vp]),
            "destroy_microenvironment": (C.c_int, [vp]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype, f.argtypes = res, args
        _lib = L
    return _lib


def _ck(rc):
    if rc != MECH_OK:
        raise MechError(rc, mech_last_error())


def _d(a):
    return None if a is None else a.ctypes.data_as(C.POINTER(C.c_double))


def mech_last_error() -> str:
    return lib().mech_last_error().decode()


def mech_abi_version() -> int:
    return int(lib().mech_abi_version())


def mech_device_count() -> int:
    return int(lib().mech_device_count())


def make_params(lo, hi, voxel_size=30.0, dt=0.1, c_rep=10.0, rel_adh_distance=1.25,
                c_adh=((0.4,),), precision=MECH_FP64, ab2_start=MECH_AB2_ZERO_HISTORY,
                flags=0) -> MechParams:
    if isinstance(precision, str):
        precision = PRECISIONS[precision]
    p = MechParams()
    p.abi_version = MECH_ABI_VERSION
    p.precision, p.ab2_start, p.flags = int(precision), int(ab2_start), int(flags)
    for a in range(3):
        p.domain_lo[a], p.domain_hi[a] = float(lo[a]), float(hi[a])
    p.voxel_size, p.dt, p.c_rep = float(voxel_size), float(dt), float(c_rep)
    p.rel_adh_distance = float(rel_adh_distance)
    c = np.asarray(c_adh, dtype=np.float64)
    p.n_types = int(c.shape[0])
    p.reserved = 0
    for k, v in enumerate(c.reshape(-1)):
        p.c_adh[k] = float(v)
    return p


def params_of(pop, precision=MECH_FP64, ab2_start=MECH_AB2_ZERO_HISTORY, flags=0) -> MechParams:
    """Parameters of a workloads.Population."""
    return make_params(pop.lo, pop.hi, pop.voxel, pop.dt, pop.c_rep, pop.alpha, pop.c_adh,
                       precision, ab2_start, flags)


def population_workspace_bytes(params: MechParams, n_cells: int) -> int:
    r = int(lib().population_workspace_bytes(C.byref(params), int(n_cells)))
    if r < 0:
        raise MechError(r, mech_last_error())
    return r


def _cells(pos, radius, type_, prev_velocity):
    pos = np.ascontiguousarray(pos, dtype=np.float64).reshape(-1, 3)
    radius = np.ascontiguousarray(radius, dtype=np.float64).reshape(-1)
    t = None if type_ is None else np.ascontiguousarray(type_, dtype=np.int32).reshape(-1)
    vp = (None if prev_velocity is None
          else np.ascontiguousarray(prev_velocity, dtype=np.float64).reshape(-1, 3))
    if radius.shape[0] != pos.shape[0] or (t is not None and t.shape[0] != pos.shape[0]) or \
            (vp is not None and vp.shape[0] != pos.shape[0]):
        raise MechError(MECH_E_INVALID, "array lengths differ")
    return pos, radius, t, vp


def create_population(params: MechParams, pos, radius, type=None, prev_velocity=None,
                      stream=None) -> C.c_void_p:
    pos, radius, t, vp = _cells(pos, radius, type, prev_velocity)
    h = C.c_void_p()
    _ck(lib().create_population(C.byref(params), pos.shape[0], _d(pos), _d(radius),
                                None if t is None else t.ctypes.data_as(C.POINTER(C.c_int32)),
                                _d(vp), stream, C.byref(h)))
    return h


def create_population_cap(params: MechParams, pos, radius, type, prev_velocity, stream,
                          max_cells: int) -> C.c_void_p:
    pos, radius, t, vp = _cells(pos, radius, type, prev_velocity)
    h = C.c_void_p()
    _ck(lib().create_population_cap(C.byref(params), pos.shape[0], int(max_cells), _d(pos),
                                    _d(radius),
                                    None if t is None else t.ctypes.data_as(C.POINTER(C.c_int32)),
                                    _d(vp), stream, C.byref(h)))
    return h


def create_population_in(params: MechParams, pos, radius, type, prev_velocity, stream,
                         workspace_ptr: int, workspace_bytes: int) -> C.c_void_p:
    pos, radius, t, vp = _cells(pos, radius, type, prev_velocity)
    h = C.c_void_p()
    _ck(lib().create_population_in(C.byref(params), pos.shape[0], _d(pos), _d(radius),
                                   None if t is None else t.ctypes.data_as(C.POINTER(C.c_int32)),
                                   _d(vp), stream, C.c_void_p(workspace_ptr),
                                   int(workspace_bytes), C.byref(h)))
    return h


def step_mechanics_noalloc(params: MechParams, pos, radius, type=None, prev_velocity=None, n_steps: int = 1,
                           stream=None):
    """create + n_steps steps + read_state in one call on the library's static scratch.
    Returns (pos, vel, interactions)."""
    pos, radius, t, vp = _cells(pos, radius, type, prev_velocity)
    n = pos.shape[0]
    out = np.empty((n, 3), np.float64)
    vel = np.empty((n, 3), np.float64)
    inter = C.c_int64(0)
    _ck(lib().step_mechanics_noalloc(C.byref(params), n, _d(pos), _d(radius),
                                     None if t is None else t.ctypes.data_as(C.POINTER(C.c_int32)),
                                     _d(vp), int(n_steps), stream, _d(out), _d(vel), C.byref(inter)))
    return out, vel, int(inter.value)


def step_mechanics(h, n_steps: int = 1) -> None:
    _ck(lib().step_mechanics(h, int(n_steps)))


def population_info(h):
    n = C.c_int64()
    dims = (C.c_int32 * 3)()
    _ck(lib().population_info(h, C.byref(n), dims))
    return int(n.value), tuple(int(x) for x in dims)


def read_state(h, with_velocity: bool = True):
    n, _ = population_info(h)
    pos = np.empty((n, 3), np.float64)
    vel = np.empty((n, 3), np.float64) if with_velocity else None
    _ck(lib().read_state(h, _d(pos), _d(vel), n))
    return pos, vel


def read_binning(h):
    n, dims = population_info(h)
    V = dims[0] * dims[1] * dims[2]
    up = lambda a: a.ctypes.data_as(C.POINTER(C.c_uint32))
    vid = np.empty(max(n, 1), np.uint32)
    start = np.empty(V + 1, np.uint32)
    ids = np.empty(max(n, 1), np.uint32)
    occ = np.empty(V, np.uint32)
    m, nv = C.c_int64(), C.c_int64()
    _ck(lib().read_binning(h, up(vid), up(start), up(ids), up(occ), C.byref(m), C.byref(nv)))
    return vid[:n], start, ids[:n], occ[:m.value]


def read_stats(h):
    s, i, c = C.c_int64(), C.c_int64(), C.c_int64()
    _ck(lib().read_stats(h, C.byref(s), C.byref(i), C.byref(c)))
    return int(s.value), int(i.value), int(c.value)


def read_xcd_split(h):
    split = np.zeros(9, np.uint32)
    _ck(lib().read_xcd_split(h, split.ctypes.data_as(C.POINTER(C.c_uint32))))
    return split


def profile_step(h, n_steps: int = 1):
    """Mean ms per step of (binning + reorder, force + update), timed with HIP events."""
    ms = np.zeros(2, np.float64)
    _ck(lib().profile_step(h, int(n_steps), _d(ms)))
    return float(ms[0]), float(ms[1])


def population_stream(h) -> int:
    return int(lib().population_stream(h) or 0)


def destroy_population(h) -> None:
    if h:
        _ck(lib().destroy_population(h))


class Population:
    """Owns one device population; `with Population(...) as p:` destroys it on exit."""

    def __init__(self, params: MechParams, pos, radius, type=None, prev_velocity=None,
                 stream=None, workspace=None, max_cells=None):
        self.n = int(np.asarray(pos).reshape(-1, 3).shape[0])
        self._ws = workspace  # keeps a caller's device buffer (e.g. a torch tensor) alive
        if max_cells is not None:
            self.h = create_population_cap(params, pos, radius, type, prev_velocity, stream,
                                           max_cells)
        elif workspace is not None:
            self.h = create_population_in(params, pos, radius, type, prev_velocity, stream,
                                          int(workspace.data_ptr()),
                                          int(workspace.numel() * workspace.element_size()))
        else:
            self.h = create_population(params, pos, radius, type, prev_velocity, stream)

    def step(self, n_steps=1):
        step_mechanics(self.h, n_steps)
        return self

    def state(self, with_velocity=True):
        return read_state(self.h, with_velocity)

    def binning(self):
        return read_binning(self.h)

    def stats(self):
        return read_stats(self.h)

    def xcd_split(self):
        return read_xcd_split(self.h)

    def profile(self, n_steps=1):
        return profile_step(self.h, n_steps)

    def set_division(self, p_div: float, seed: int = 0):
        """Cells divide with probability p_div per step (the population needs max_cells)."""
        _ck(lib().population_set_division(self.h, float(p_div), C.c_uint64(seed)))

    def set_death(self, p_death: float):
        """Cells die with probability p_death per step, after division (draws from the
        division seed's stream with its top bit flipped)."""
        _ck(lib().population_set_death(self.h, float(p_death)))

    def size(self) -> int:
        n = C.c_int64()
        _ck(lib().population_size(self.h, C.byref(n)))
        return int(n.value)

    def set_reorder(self, every: int):
        """Reorder the cells every `every` steps (1: every step); 0: never, cells in id
        order (the locality study)."""
        _ck(lib().population_set_reorder(self.h, int(every)))

    def get_tuning(self) -> MechTuning:
        t = MechTuning()
        _ck(lib().population_get_tuning(self.h, C.byref(t)))
        return t

    def set_tuning(self, t: MechTuning):
        _ck(lib().population_set_tuning(self.h, C.byref(t)))

    @property
    def stream(self) -> int:
        return population_stream(self.h)

    def close(self):
        if self.h:
            destroy_population(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------------------- batches

def batch_workspace_bytes(params: MechParams, max_cells: int, max_voxels: int,
                          max_slots: int) -> int:
    r = int(lib().batch_workspace_bytes(C.byref(params), int(max_cells), int(max_voxels),
                                        int(max_slots)))
    if r < 0:
        raise MechError(r, mech_last_error())
    return r


def batch_request_voxels(params: MechParams, lo, hi) -> int:
    lo = np.ascontiguousarray(lo, dtype=np.float64)
    hi = np.ascontiguousarray(hi, dtype=np.float64)
    r = int(lib().batch_request_voxels(C.byref(params), _d(lo), _d(hi)))
    if r < 0:
        raise MechError(r, mech_last_error())
    return r


def batch_budget_capacity(params: MechParams, budget_bytes: int, voxels_per_cell: float,
                          max_slots: int):
    """(max_cells, max_voxels) of the largest arena within the budget (computed by the
    library on the host; no device needed)."""
    c, v = C.c_int64(), C.c_int64()
    _ck(lib().batch_budget_capacity(C.byref(params), int(budget_bytes), float(voxels_per_cell),
                                    int(max_slots), C.byref(c), C.byref(v)))
    return int(c.value), int(v.value)


def batch_sync(batch) -> None:
    """Wait until every step enqueued on the batch has completed."""
    _ck(lib().batch_sync(batch.h))


class Batch:
    """Many independent simulations advanced together (see include/mech.h)."""

    def __init__(self, params: MechParams, max_cells: int = 0, max_voxels: int = 1,
                 max_slots: int = 1, stream=None, workspace=None, budget_bytes=None,
                 voxels_per_cell: float = 1.6):
        """Capacity given as max_cells/max_voxels/max_slots, or (budget_bytes set) sized
        by the library from an HBM byte budget for max_slots slots."""
        self.params = params
        self._ws = workspace
        h = C.c_void_p()
        if budget_bytes is not None:
            _ck(lib().create_batch_budget(C.byref(params), int(budget_bytes), float(voxels_per_cell),
                                          int(max_slots), stream, C.byref(h)))
        elif workspace is not None:
            _ck(lib().create_batch_in(C.byref(params), int(max_cells), int(max_voxels),
                                      int(max_slots), stream, C.c_void_p(int(workspace.data_ptr())),
                                      int(workspace.numel() * workspace.element_size()),
                                      C.byref(h)))
        else:
            _ck(lib().create_batch(C.byref(params), int(max_cells), int(max_voxels),
                                   int(max_slots), stream, C.byref(h)))
        self.h = h
        self.max_slots = int(max_slots)
        self.sizes = {}

    def admit(self, lo, hi, pos, radius, type=None, prev_velocity=None, n_steps=-1) -> int:
        pos, radius, t, vp = _cells(pos, radius, type, prev_velocity)
        lo = np.ascontiguousarray(lo, dtype=np.float64)
        hi = np.ascontiguousarray(hi, dtype=np.float64)
        slot = C.c_int32(-1)
        _ck(lib().batch_admit(self.h, _d(lo), _d(hi), pos.shape[0], _d(pos), _d(radius),
                              None if t is None else t.ctypes.data_as(C.POINTER(C.c_int32)),
                              _d(vp), int(n_steps), C.byref(slot)))
        self.sizes[slot.value] = pos.shape[0]
        return slot.value

    def admit_pop(self, pop, n_steps=None, prev_velocity=None) -> int:
        return self.admit(pop.lo, pop.hi, pop.pos, pop.radius, pop.type, prev_velocity,
                          pop.steps if n_steps is None else n_steps)

    def step(self, n_steps=1):
        _ck(lib().batch_step(self.h, int(n_steps)))
        return self

    def sync(self):
        """Wait until every step enqueued on the batch has completed."""
        _ck(lib().batch_sync(self.h))

    def capacity(self):
        c, v, b = C.c_int64(), C.c_int64(), C.c_int64()
        s = C.c_int32()
        _ck(lib().batch_capacity(self.h, C.byref(c), C.byref(v), C.byref(s), C.byref(b)))
        return dict(max_cells=c.value, max_voxels=v.value, max_slots=s.value, arena_bytes=b.value)

    def mark_clock(self):
        """Zero of done_ms: recorded on the stream and waited for."""
        _ck(lib().batch_mark_clock(self.h))

    def done_ms(self, slot) -> float:
        """Device ms from mark_clock to the completion of the slot's last step."""
        ms = C.c_double()
        _ck(lib().batch_slot_done_ms(self.h, int(slot), C.byref(ms)))
        return float(ms.value)

    def poll(self):
        out = np.zeros(self.max_slots, np.int32)
        n = C.c_int32(0)
        _ck(lib().batch_poll(self.h, out.ctypes.data_as(C.POINTER(C.c_int32)), self.max_slots,
                             C.byref(n)))
        return [int(x) for x in out[:n.value]]

    def read(self, slot, with_velocity=True):
        n = self.sizes[slot]
        pos = np.empty((n, 3), np.float64)
        vel = np.empty((n, 3), np.float64) if with_velocity else None
        _ck(lib().batch_read(self.h, int(slot), _d(pos), _d(vel), n))
        return pos, vel

    def retire(self, slot):
        _ck(lib().batch_retire(self.h, int(slot)))
        self.sizes.pop(slot, None)

    def slot_info(self, slot):
        n, s = C.c_int64(), C.c_int64()
        _ck(lib().batch_slot_info(self.h, int(slot), C.byref(n), C.byref(s)))
        return int(n.value), int(s.value)

    def info(self):
        a, b, fc, fv = C.c_int64(), C.c_int64(), C.c_int64(), C.c_int64()
        nl = C.c_int32()
        _ck(lib().batch_info(self.h, C.byref(a), C.byref(b), C.byref(nl), C.byref(fc), C.byref(fv)))
        return dict(n_cells=a.value, n_voxels=b.value, n_live=nl.value, free_cells=fc.value,
                    free_voxels=fv.value)

    def stats(self):
        s, i, c = C.c_int64(), C.c_int64(), C.c_int64()
        _ck(lib().batch_stats(self.h, C.byref(s), C.byref(i), C.byref(c)))
        return int(s.value), int(i.value), int(c.value)

    def profile(self, n_steps=1):
        ms = np.zeros(2, np.float64)
        _ck(lib().batch_profile(self.h, int(n_steps), _d(ms)))
        return float(ms[0]), float(ms[1])

    def set_flags(self, flags: int):
        _ck(lib().batch_set_flags(self.h, int(flags)))
        self.params.flags = int(flags)

    def get_tuning(self) -> MechTuning:
        t = MechTuning()
        _ck(lib().batch_get_tuning(self.h, C.byref(t)))
        return t

    def set_tuning(self, t: MechTuning):
        _ck(lib().batch_set_tuning(self.h, C.byref(t)))
        self.params.flags = (int(self.params.flags) & ~MECH_FORCE_KERNEL_MASK) | int(t.force_kernel)

    @property
    def stream(self) -> int:
        return int(lib().batch_stream(self.h) or 0)

    def close(self):
        if getattr(self, "h", None):
            _ck(lib().destroy_batch(self.h))
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------- microenvironment

def microenv_params(dims, voxel_size=20.0, dt=0.01, diffusion=(1e5,), decay=(0.1,)) -> MechMicroenvParams:
    p = MechMicroenvParams()
    p.abi_version = MECH_ABI_VERSION
    D = np.atleast_1d(np.asarray(diffusion, dtype=np.float64))
    lam = np.atleast_1d(np.asarray(decay, dtype=np.float64))
    if D.shape != lam.shape:
        raise ValueError("diffusion and decay need one value per substrate")
    p.n_substrates = int(D.size)
    for a in range(3):
        p.dims[a] = int(dims[a])
    p.voxel_size, p.dt = float(voxel_size), float(dt)
    for k in range(min(D.size, MECH_MAX_SUBSTRATES)):
        p.diffusion[k] = float(D[k])
        p.decay[k] = float(lam[k])
    return p


def microenv_params_of(env) -> MechMicroenvParams:
    """From a workloads.Microenv description."""
    return microenv_params(env.dims, env.dx, env.dt, env.diffusion, env.decay)


class Microenv:
    """A substrate mesh on the device (create_microenvironment ... destroy)."""

    def __init__(self, params: MechMicroenvParams, density=None, stream=None):
        self.params = params
        nx, ny, nz = (int(params.dims[a]) for a in range(3))
        self.shape = (int(params.n_substrates), nz, ny, nx)
        self.n_values = int(np.prod(self.shape))
        rho = None
        if density is not None:
            rho = np.ascontiguousarray(density, dtype=np.float64).reshape(-1)
            if rho.size != self.n_values:
                raise ValueError(f"density holds {rho.size} values, the mesh {self.n_values}")
        h = C.c_void_p()
        _ck(lib().create_microenvironment(C.byref(params), _d(rho), stream, C.byref(h)))
        self.h = h

    def step(self, n_steps=1):
        _ck(lib().microenvironment_step(self.h, int(n_steps)))

    def compute_gradients(self):
        _ck(lib().microenvironment_gradients(self.h))

    def density(self):
        out = np.empty(self.n_values, np.float64)
        _ck(lib().read_density(self.h, _d(out), out.size))
        return out.reshape(self.shape)

    def gradients(self):
        out = np.empty(3 * self.n_values, np.float64)
        _ck(lib().read_gradients(self.h, _d(out), out.size))
        s, nz, ny, nx = self.shape
        return out.reshape(s, 3, nz, ny, nx)

    def set_density(self, density):
        rho = np.ascontiguousarray(density, dtype=np.float64).reshape(-1)
        _ck(lib().write_density(self.h, _d(rho), rho.size))

    def profile(self, n_steps=1):
        """Mean ms per launch of the x, y and z solves and of the gradient kernel."""
        ms = np.zeros(4, np.float64)
        _ck(lib().microenvironment_profile(self.h, int(n_steps), _d(ms)))
        return tuple(float(x) for x in ms)

    def device_arrays(self):
        d, g = C.c_void_p(), C.c_void_p()
        _ck(lib().microenvironment_device_arrays(self.h, C.byref(d), C.byref(g)))
        return d.value, g.value

    @property
    def stream(self) -> int:
        return int(lib().microenvironment_stream(self.h) or 0)

    def close(self):
        if getattr(self, "h", None):
            h, self.h = self.h, None
            _ck(lib().destroy_microenvironment(h))

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
