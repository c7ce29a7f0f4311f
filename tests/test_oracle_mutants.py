"""The oracle's pins catch plausible mistakes.

Each mutant is a copy of oracle/mech_oracle.c (or oracle/diffusion_oracle.c) with one
mistake planted: a dropped term, a wrong sign, a wrong index, an off-by-one, a wrong
tie-break, a wrong boundary row.  The copy is compiled on the CPU and the oracle's pin
tests are run against it in a child process (through MECH_ORACLE_LIB or
DIFF_ORACLE_LIB); at least one pin must fail.  The mutants never leave the CPU.
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

import pytest

import oracle
from oracle import diffusion as OD

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "mech_oracle.c")
PINS = ["tests/test_oracle_closed_form.py", "tests/test_oracle_invariants.py", "tests/test_oracle_fp32.py",
        "tests/test_oracle_bruteforce.py", "tests/test_oracle_binning.py", "tests/test_kahan.py",
        "tests/test_oracle_division.py", "tests/test_oracle_death.py"]

# (name, text in mech_oracle.c, replacement); each text occurs exactly once
MUTANTS = [
    ("repulsion sign",
     "        w += p->c_rep * u * u;", "        w -= p->c_rep * u * u;"),
    ("adhesion dropped",
     "    w -= p->c_adh[ti * p->n_types + tj] * a * a;\n    double s", "    double s"),
    ("adhesion matrix index",
     "    w -= p->c_adh[ti * p->n_types + tj] * a * a;\n    double s",
     "    w -= p->c_adh[ti * p->n_types + ti] * a * a;\n    double s"),
    ("adhesion distance without alpha",
     "    double RA = p->alpha * R;", "    double RA = R;"),
    ("repulsion cutoff at R_A",
     "    double w = 0.0;\n    if (d < R) {", "    double w = 0.0;\n    if (d < RA) {"),
    ("force direction on one axis",
     "    acc[0] += s * dx;", "    acc[0] -= s * dx;"),
    ("coincident cells not skipped",
     "    if (!(d2 > 0.0 && d2 < RA * RA)) return 0;", "    if (!(d2 < RA * RA)) return 0;"),
    ("Adams-Bashforth weight sign",
     "(1.5 * v - 0.5 * vp)", "(1.5 * v + 0.5 * vp)"),
    ("Euler start ignored",
     "double vp = euler_start ? v : vprev[3 * i + c];", "double vp = vprev[3 * i + c];"),
    ("upper wall clamps instead of mirroring",
     "    if (x > hi) x = 2.0 * hi - x;", "    if (x > hi) x = hi;"),
    ("neighbour voxels on one side only",
     "        memset(&accf, 0, sizeof accf);\n        for (int dz = -1; dz <= 1; ++dz)\n"
     "            for (int dy = -1; dy <= 1; ++dy)\n                for (int dx = -1; dx <= 1; ++dx) {",
     "        memset(&accf, 0, sizeof accf);\n        for (int dz = -1; dz <= 1; ++dz)\n"
     "            for (int dy = -1; dy <= 1; ++dy)\n                for (int dx = -1; dx <= 0; ++dx) {"),
    ("voxel numbering y fastest",
     "    return k[0] + (int64_t)dims[0] * (k[1] + (int64_t)dims[1] * k[2]);",
     "    return k[1] + (int64_t)dims[1] * (k[0] + (int64_t)dims[0] * k[2]);"),
    ("a cell on a voxel face binned into the voxel below",
     "        double f = floor((x[a] - p->lo[a]) * inv_h);",
     "        double f = ceil((x[a] - p->lo[a]) * inv_h) - 1.0;"),
    ("ties broken by descending id",
     "    for (int64_t i = 0; i < n; ++i) sorted_ids[cursor[vid[i]]++] = (uint32_t)i;",
     "    for (int64_t i = n - 1; i >= 0; --i) sorted_ids[cursor[vid[i]]++] = (uint32_t)i;"),
    ("occupied voxels named one voxel late",
     "        if (voxel_start[v + 1] > voxel_start[v]) occ[m++] = (uint32_t)v;",
     "        if (voxel_start[v + 1] > voxel_start[v]) occ[m++] = (uint32_t)(v + 1);"),
    ("scan drops the last voxel",
     "    for (int64_t v = 0; v < V; ++v) voxel_start[v + 1] += voxel_start[v];",
     "    for (int64_t v = 0; v + 1 < V; ++v) voxel_start[v + 1] += voxel_start[v];"),
    ("empty voxels listed as occupied",
     "        if (voxel_start[v + 1] > voxel_start[v]) occ[m++]",
     "        if (voxel_start[v + 1] >= voxel_start[v]) occ[m++]"),
    ("Kahan compensation sign",
     "        *c = (t - *sum) - y;", "        *c = (t - *sum) + y;"),
    ("float distance without its z term",
     "    float d2 = dx * dx + dy * dy + dz * dz;", "    float d2 = dx * dx + dy * dy;"),
    ("float distance fused",
     "    float d2 = dx * dx + dy * dy + dz * dz;", "    float d2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));"),
    ("float repulsion dropped",
     "        w += (float)p->c_rep * u * u;", "        w += 0.0f;"),
    ("division draw from the direction counter",
     "oracle_uniform(seed, (uint64_t)id, (uint64_t)t, 0) < p_div",
     "oracle_uniform(seed, (uint64_t)id, (uint64_t)t, 1) < p_div"),
    ("daughter placed on the parent's side",
     "pos[3 * q + c] = reflect(x + half * e[c]", "pos[3 * q + c] = reflect(x - half * e[c]"),
    ("daughters a full radius away",
     "    double half = 0.5 * radius[id];", "    double half = radius[id];"),
    ("capacity filled from the highest id",
     "    for (int64_t id = 0; id < n && n + made < capacity; ++id) {",
     "    for (int64_t id = n - 1; id >= 0 && n + made < capacity; --id) {"),
    ("death drawn from the division stream",
     "    const uint64_t seed_d = seed ^ 0x8000000000000000ull;", "    const uint64_t seed_d = seed;"),
    ("the drawn cells survive instead of dying",
     "        if (oracle_uniform(seed_d, (uint64_t)id, (uint64_t)t, 0) < p_death) continue;",
     "        if (!(oracle_uniform(seed_d, (uint64_t)id, (uint64_t)t, 0) < p_death)) continue;"),
    ("a survivor's type left behind",
     "            radius[kept] = radius[id];\n            type[kept] = type[id];",
     "            radius[kept] = radius[id];"),
]


DIFF_SRC = os.path.join(ROOT, "oracle", "diffusion_oracle.c")
DIFF_PINS = ["tests/test_oracle_diffusion.py"]

# (name, text in diffusion_oracle.c, replacement); each text occurs exactly once
DIFF_MUTANTS = [
    ("first face row without the no-flux correction",
     "    double diag = b + r;\n    cp[0]", "    double diag = b + 2.0 * r;\n    cp[0]"),
    ("last face row without the no-flux correction",
     "        diag = (i == n - 1) ? b + r : b + 2.0 * r;", "        diag = b + 2.0 * r;"),
    ("decay not split over the three sweeps",
     "        const double b = 1.0 + p->decay[s] * p->dt / 3.0;",
     "        const double b = 1.0 + p->decay[s] * p->dt;"),
    ("diffusion number over dx instead of dx^2",
     "p->diffusion[s] * p->dt / (p->dx * p->dx);", "p->diffusion[s] * p->dt / p->dx;"),
    ("back substitution sign",
     "        u[i * stride] = u[i * stride] - cp[i] * u[(i + 1) * stride];",
     "        u[i * stride] = u[i * stride] + cp[i] * u[(i + 1) * stride];"),
    ("first substrate's coefficients for all",
     "        const double r = p->diffusion[s] *", "        const double r = p->diffusion[0] *"),
    ("sweeps in reverse order",
     "        sweep(p, rho, 0);\n        sweep(p, rho, 1);\n        sweep(p, rho, 2);",
     "        sweep(p, rho, 2);\n        sweep(p, rho, 1);\n        sweep(p, rho, 0);"),
    ("central difference over dx",
     "else val = (u[v + st] - u[v - st]) / (2.0 * p->dx);", "else val = (u[v + st] - u[v - st]) / p->dx;"),
    ("first-face gradient halved",
     "else if (c == 0) val = (u[v + st] - u[v]) / p->dx;",
     "else if (c == 0) val = (u[v + st] - u[v]) / (2.0 * p->dx);"),
    ("gradient y stride from the wrong axis",
     "    const int64_t stride[3] = {1, nx, (int64_t)nx * ny};",
     "    const int64_t stride[3] = {1, ny, (int64_t)nx * ny};"),
]


def _run_pins(name, text, repl, workdir, src_path=SRC, pins=PINS, var="MECH_ORACLE_LIB",
              compile_to=oracle.compile_to):
    src = open(src_path).read()
    assert src.count(text) == 1, f"mutant '{name}': its text is not unique in {src_path}"
    tag = "".join(ch if ch.isalnum() else "_" for ch in name)
    c_path = os.path.join(workdir, f"mutant_{tag}.c")
    so_path = os.path.join(workdir, f"mutant_{tag}.so")
    with open(c_path, "w") as f:
        f.write(src.replace(text, repl))
    compile_to(c_path, so_path)
    env = dict(os.environ, OMP_NUM_THREADS="2")
    env[var] = so_path
    res = subprocess.run([sys.executable, "-m", "pytest", *pins, "-x", "-q", "-m", "not gpu",
                          "-p", "no:cacheprovider"], cwd=ROOT, env=env, capture_output=True,
                         text=True, timeout=600)
    return res.returncode, res.stdout[-600:]


def _run_diff_pins(name, text, repl, workdir):
    return _run_pins(name, text, repl, workdir, DIFF_SRC, DIFF_PINS, "DIFF_ORACLE_LIB",
                     OD.compile_to)


def test_every_mutant_fails_a_pin(tmp_path):
    with ThreadPoolExecutor(max_workers=4) as ex:
        futs = {name: ex.submit(_run_pins, name, text, repl, str(tmp_path))
                for name, text, repl in MUTANTS}
        results = {name: f.result() for name, f in futs.items()}
    survivors = [name for name, (rc, _) in results.items() if rc == 0]
    assert not survivors, f"mutants no pin caught: {survivors}"
    # rc 1 = tests failed; anything else would be a crash of the run itself
    crashed = {name: out for name, (rc, out) in results.items() if rc not in (0, 1)}
    assert not crashed, crashed


def test_unmutated_copy_passes_the_pins(tmp_path):
    rc, out = _run_pins("identity", "#include <math.h>", "#include <math.h>", str(tmp_path))
    assert rc == 0, out


@pytest.mark.parametrize("name,text,repl", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_mutant_text_is_present(name, text, repl):
    assert open(SRC).read().count(text) == 1


def test_every_diffusion_mutant_fails_a_pin(tmp_path):
    with ThreadPoolExecutor(max_workers=4) as ex:
        futs = {name: ex.submit(_run_diff_pins, name, text, repl, str(tmp_path))
                for name, text, repl in DIFF_MUTANTS}
        results = {name: f.result() for name, f in futs.items()}
    survivors = [name for name, (rc, _) in results.items() if rc == 0]
    assert not survivors, f"mutants no pin caught: {survivors}"
    crashed = {name: out for name, (rc, out) in results.items() if rc not in (0, 1)}
    assert not crashed, crashed


def test_unmutated_diffusion_copy_passes_the_pins(tmp_path):
    rc, out = _run_diff_pins("identity", "#include <math.h>", "#include <math.h>", str(tmp_path))
    assert rc == 0, out


@pytest.mark.parametrize("name,text,repl", DIFF_MUTANTS, ids=[m[0] for m in DIFF_MUTANTS])
def test_diffusion_mutant_text_is_present(name, text, repl):
    assert open(DIFF_SRC).read().count(text) == 1
