"""Seeded synthetic inputs for the mechanics step (shared by the oracle and the GPU path).

This module only draws numbers: it holds none of the method's arithmetic (no binning,
no force law, no integration).  Both the CPU oracle and the HIP library receive the
arrays built here, so the two sides always start from identical inputs.

The paper's own workload (the 3D "heterogeneity" sample project: a little over 3900
initial cells in a 1500 um box, Section 3.2) is not available; the spheroids below are
synthetic stand-ins with the shapes, sizes and value distributions of the five
workloads the mechanics step is benchmarked on:

  plain1k   1,000 cells uniform in a 200 um cube, radius 8.4 um, one type, 100 steps
  sph100k   100,000 cells uniform in a ball at ~0.6 volume fraction, radii N(8.4, 0.5)
            clipped to [6, 11], two types with a 2x2 adhesion matrix, 1,000 steps
  tumour1m  1,000,000 cells in a 2 mm cube: 900k in a 600 um ball + 100k uniform,
            radii as sph100k, one type, 200 steps
  batch256  256 independent sph100k-like spheroids, sizes log-uniform in [1k, 100k]
  serve     Poisson request stream, sizes log-uniform in [1k, 500k], steps U{10..1000}
  env75     substrate mesh of the microenvironment solver: 75 x 75 x 75 voxels of 20 um
            (the paper's 75^3 mesh over the 1500 um box of its sample project), an
            oxygen-like substrate (D = 1e5 um^2/min, decay 0.1 /min), dt = 0.01 min;
            further substrates draw D and decay log-uniformly; densities are a seeded
            smooth field plus white noise

Draw order for every population: radii, then types, then positions.  Ball positions
are drawn by rejection from the bounding cube.  Generator: numpy PCG64.
"""
from __future__ import annotations

import hashlib
import math
from dataclasses import dataclass, field

import numpy as np

VOXEL = 30.0          # mechanics voxel edge, um
DT = 0.1              # min
C_REP = 10.0
ALPHA = 1.25          # adhesion distance = ALPHA * (r_i + r_j)
R_MEAN, R_SD, R_MIN, R_MAX = 8.4, 0.5, 6.0, 11.0
C_ADH_1 = [[0.4]]
C_ADH_2 = [[0.4, 0.1], [0.1, 0.4]]


@dataclass
class Population:
    """One simulation's inputs: positions (n,3) f64, radii (n,) f64, types (n,) i32."""
    name: str
    pos: np.ndarray
    radius: np.ndarray
    type: np.ndarray
    lo: tuple
    hi: tuple
    c_adh: list
    steps: int
    voxel: float = VOXEL
    dt: float = DT
    c_rep: float = C_REP
    alpha: float = ALPHA
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.pos.shape[0])

    @property
    def n_types(self) -> int:
        return len(self.c_adh)

    @property
    def half_width(self) -> float:
        """Domain half-width S, the scale of the position-error metric."""
        return 0.5 * max(h - l for l, h in zip(self.lo, self.hi))

    def sha256(self) -> str:
        m = hashlib.sha256()
        for a in (self.pos, self.radius, self.type):
            m.update(np.ascontiguousarray(a).tobytes())
        return m.hexdigest()


def _radii(rng: np.random.Generator, n: int) -> np.ndarray:
    return np.clip(rng.normal(R_MEAN, R_SD, n), R_MIN, R_MAX).astype(np.float64)


def _uniform_cube(rng, n, lo, hi):
    return rng.uniform(lo, hi, size=(n, 3)).astype(np.float64)


def _uniform_ball(rng, n, radius):
    out = np.empty((n, 3), dtype=np.float64)
    got = 0
    while got < n:
        need = n - got
        cand = rng.uniform(-radius, radius, size=(int(need * 2.0) + 64, 3))
        keep = cand[np.einsum("ij,ij->i", cand, cand) <= radius * radius]
        take = min(need, keep.shape[0])
        out[got:got + take] = keep[:take]
        got += take
    return out


def _spheroid_domain(r_ball: float) -> float:
    """Half-width of the cube around a ball: a whole number of voxels, 1.5x the ball."""
    return VOXEL * math.ceil(1.5 * r_ball / VOXEL)


def plain(n: int = 1000, seed: int = 1, steps: int = 100, half: float = 100.0) -> Population:
    """Uniform cells in a cube that is also the domain; one type; radius 8.4 um."""
    rng = np.random.Generator(np.random.PCG64(seed))
    radius = np.full(n, R_MEAN, dtype=np.float64)
    types = np.zeros(n, dtype=np.int32)
    pos = _uniform_cube(rng, n, -half, half)
    lo, hi = (-half,) * 3, (half,) * 3
    return Population(f"plain{n}", pos, radius, types, lo, hi, C_ADH_1, steps)


def spheroid(n: int = 100_000, seed: int = 2, steps: int = 1000, phi: float = 0.6,
             two_types: bool = True) -> Population:
    """Cells uniform in a ball whose radius puts the sphere-volume fraction at phi."""
    rng = np.random.Generator(np.random.PCG64(seed))
    radius = _radii(rng, n)
    if two_types:
        types = (rng.random(n) < 0.5).astype(np.int32)
        c_adh = C_ADH_2
    else:
        types = np.zeros(n, dtype=np.int32)
        c_adh = C_ADH_1
    r_ball = float(np.cbrt(np.sum(radius ** 3) / phi))
    pos = _uniform_ball(rng, n, r_ball)
    w = _spheroid_domain(r_ball)
    return Population(f"sph{n}", pos, radius, types, (-w,) * 3, (w,) * 3, c_adh, steps,
                      meta={"r_ball": r_ball})


def tumour(n: int = 1_000_000, seed: int = 3, steps: int = 200, core_frac: float = 0.9,
           core_radius: float = 600.0, half: float = 1000.0) -> Population:
    """Dense ball core plus uniformly scattered cells in a 2*half cube; one type."""
    rng = np.random.Generator(np.random.PCG64(seed))
    radius = _radii(rng, n)
    types = np.zeros(n, dtype=np.int32)
    n_core = int(round(core_frac * n))
    pos = np.concatenate([_uniform_ball(rng, n_core, core_radius),
                          _uniform_cube(rng, n - n_core, -half, half)])
    return Population(f"tumour{n}", pos, radius, types, (-half,) * 3, (half,) * 3, C_ADH_1,
                      steps, meta={"core_radius": core_radius, "n_core": n_core})


def batch_sizes(n_sims: int = 256, seed: int = 4000, lo: float = 1e3, hi: float = 1e5):
    rng = np.random.Generator(np.random.PCG64(seed))
    return [int(math.floor(math.exp(rng.uniform(math.log(lo), math.log(hi)))))
            for _ in range(n_sims)]


def batch(n_sims: int = 256, steps: int = 500, size_hi: float = 1e5):
    """Independent spheroids of log-uniform size; simulation k uses seed 4000 + k."""
    sizes = batch_sizes(n_sims, 4000, 1e3, size_hi)
    return [spheroid(n, seed=4000 + k, steps=steps) for k, n in enumerate(sizes)]


@dataclass
class Request:
    rid: int
    arrival_s: float
    n: int
    steps: int
    seed: int


def request_stream(n_req: int, rate_per_s: float = 50.0, seed: int = 5,
                   size_lo: float = 1e3, size_hi: float = 5e5, steps_lo: int = 10,
                   steps_hi: int = 1000):
    """Poisson arrivals; request k's population is spheroid(n_k, seed 5000 + k)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    t = 0.0
    out = []
    for k in range(n_req):
        t += rng.exponential(1.0 / rate_per_s)
        n = int(math.floor(math.exp(rng.uniform(math.log(size_lo), math.log(size_hi)))))
        steps = int(rng.integers(steps_lo, steps_hi + 1))
        out.append(Request(k, t, n, steps, 5000 + k))
    return out


def request_population(req: Request) -> Population:
    return spheroid(req.n, seed=req.seed, steps=req.steps)


def config(name: str) -> Population:
    """The named single-simulation workloads at their full sizes."""
    if name == "plain1k":
        return plain()
    if name == "sph100k":
        return spheroid()
    if name == "tumour1m":
        return tumour()
    raise KeyError(name)


@dataclass
class Microenv:
    """A substrate mesh's inputs: dims (nx, ny, nz), voxel edge dx (um), time step dt
    (min), per-substrate diffusion (um^2/min) and decay (1/min), densities
    (n_substrates, nz, ny, nx) f64, and the step count of the workload."""
    name: str
    dims: tuple
    dx: float
    dt: float
    diffusion: tuple
    decay: tuple
    density: np.ndarray
    steps: int

    @property
    def n_substrates(self) -> int:
        return len(self.diffusion)

    @property
    def voxels(self) -> int:
        return int(np.prod(self.dims))


def microenv(dims=(75, 75, 75), n_substrates: int = 1, seed: int = 6, steps: int = 100,
             dx: float = 20.0, dt: float = 0.01) -> Microenv:
    """Substrate 0 is oxygen-like (D = 1e5 um^2/min, decay 0.1 /min); substrate k >= 1 has
    D = 10^U(2, 5) and decay 10^U(-3, 0).  Each density is 38 (0.6 + 0.4 u), u a sum of
    eight random cosine modes of wavenumber 0..4 per axis rescaled to [0, 1], plus 5%
    uniform noise (so the field holds every spatial frequency of the mesh)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    D = [1e5] + [float(10.0 ** rng.uniform(2.0, 5.0)) for _ in range(n_substrates - 1)]
    lam = [0.1] + [float(10.0 ** rng.uniform(-3.0, 0.0)) for _ in range(n_substrates - 1)]
    nx, ny, nz = dims
    ax = [(np.arange(n) + 0.5) / n for n in (nz, ny, nx)]
    rho = np.empty((n_substrates, nz, ny, nx), np.float64)
    for s in range(n_substrates):
        f = np.zeros((nz, ny, nx))
        for _ in range(8):
            k = rng.integers(0, 5, 3)
            ph = rng.uniform(0, 2 * np.pi, 3)
            f += (np.cos(np.pi * k[0] * ax[0] + ph[0])[:, None, None]
                  * np.cos(np.pi * k[1] * ax[1] + ph[1])[None, :, None]
                  * np.cos(np.pi * k[2] * ax[2] + ph[2])[None, None, :])
        f = (f - f.min()) / max(f.max() - f.min(), 1e-300)
        u = 0.95 * f + 0.05 * rng.random((nz, ny, nx))
        rho[s] = 38.0 * (0.6 + 0.4 * u)
    return Microenv(f"env{nx}x{ny}x{nz}s{n_substrates}", tuple(dims), dx, dt, tuple(D), tuple(lam),
                    rho, steps)
