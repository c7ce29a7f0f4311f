"""C-ABI checks that need no GPU: the library loads, exports every symbol that
include/mech.h declares, and rejects bad arguments on the host before touching a device."""
import ctypes as C
import os
import re
import subprocess

import numpy as np
import pytest

import workloads
from paper_2306_11544_amd import binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions(header="mech.h"):
    text = open(os.path.join(ROOT, "include", header)).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b([a-z_][a-z0-9_]*)\s*\(", text)) -
                  {"sizeof", "defined", "if", "return"})


def test_header_declares_what_binding_exports():
    assert declared_functions() == sorted(B.EXPORTS)


def test_library_exports_every_declared_symbol():
    lib = B.lib()
    for name in declared_functions():
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", B.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    syms = {line.split()[-1] for line in out.splitlines() if line.strip()}
    for name in declared_functions():
        assert name in syms, name


def test_microenv_header_declares_what_binding_exports_and_library_exports_it():
    assert declared_functions("microenv.h") == sorted(B.MICROENV_EXPORTS)
    lib = B.lib()
    out = subprocess.run(["nm", "-D", "--defined-only", B.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    syms = {line.split()[-1] for line in out.splitlines() if line.strip()}
    for name in B.MICROENV_EXPORTS:
        assert hasattr(lib, name) and name in syms, name
    # the library's internal error hook is not exported
    assert not any("report_error" in x for x in syms)


def test_microenv_params_struct_matches_header_layout():
    # 6 int32 + 2 double + 2 x 16 double
    assert C.sizeof(B.MechMicroenvParams) == 24 + 16 + 256
    assert B.MechMicroenvParams.voxel_size.offset == 24
    assert B.MechMicroenvParams.decay.offset == 24 + 16 + 128


@pytest.mark.parametrize("change", [
    {"n_substrates": 0}, {"n_substrates": 17}, {"dims": (0, 4, 4)}, {"dims": (4097, 1, 1)},
    {"dims": (2048, 2048, 1024)}, {"voxel_size": 0.0}, {"dt": -1.0}, {"reserved": 1},
    {"abi_version": 1}, {"diffusion": -1.0}, {"decay": float("nan")}])
def test_microenv_rejects_bad_parameters_on_the_host(change):
    p = B.microenv_params((8, 6, 4), diffusion=(1e3,), decay=(0.1,))
    for k, v in change.items():
        if k == "dims":
            for a in range(3):
                p.dims[a] = v[a]
        elif k in ("diffusion", "decay"):
            getattr(p, k)[0] = v
        else:
            setattr(p, k, v)
    h = C.c_void_p()
    rc = B.lib().create_microenvironment(C.byref(p), None, None, C.byref(h))
    assert rc == B.MECH_E_INVALID, B.mech_last_error()
    assert not h.value


def test_microenv_rejects_a_nonfinite_density_on_the_host():
    p = B.microenv_params((3, 2, 2), diffusion=(1e3,), decay=(0.1,))
    rho = np.zeros(12)
    rho[7] = np.inf
    h = C.c_void_p()
    rc = B.lib().create_microenvironment(C.byref(p), B._d(rho), None, C.byref(h))
    assert rc == B.MECH_E_INVALID and "density[7]" in B.mech_last_error()


def test_params_struct_matches_header_layout():
    # 4 int32 + 6 double + 4 double + 2 int32 + 64 double
    assert C.sizeof(B.MechParams) == 16 + 48 + 32 + 8 + 512
    assert B.MechParams.c_adh.offset == 16 + 48 + 32 + 8


def test_tuning_struct_matches_header_layout():
    assert C.sizeof(B.MechTuning) == 20
    t = B.tuning("voxel", 8, 2, 16, 32)
    assert t.as_dict() == {"force_kernel": B.MECH_FLAG_VOXEL_FORCE, "block_waves": 8, "unroll": 2,
                           "blocks_per_cu": 16, "list_len": 32}


def test_tuning_search_space_is_valid():
    from paper_2306_11544_amd import autotune as A
    space = A.search_space()
    assert len({tuple(t.as_dict().values()) for t in space}) == len(space)
    for t in space:
        assert t.force_kernel in (0, B.MECH_FLAG_SIMPLE_FORCE, B.MECH_FLAG_VOXEL_FORCE, B.MECH_FLAG_PRUNED_FORCE)
        assert t.block_waves in (1, 2, 4, 8) and t.unroll in (2, 4, 8)
        assert 0 <= t.blocks_per_cu <= 64
        assert t.list_len in (0, 16, 32, 64) and 2 * t.unroll <= (t.list_len or 16)


def test_tuning_calls_reject_null_handles():
    assert B.lib().population_set_reorder(None, 1) == B.MECH_E_INVALID
    t = B.tuning()
    assert B.lib().batch_set_tuning(None, C.byref(t)) == B.MECH_E_INVALID
    assert B.lib().population_get_tuning(None, C.byref(t)) == B.MECH_E_INVALID


def test_abi_version():
    assert B.mech_abi_version() == B.MECH_ABI_VERSION


def _p(**kw):
    pop = workloads.plain(10)
    return B.params_of(pop, **kw), pop


@pytest.mark.parametrize("mutate,code", [
    (lambda p: setattr(p, "abi_version", 99), B.MECH_E_INVALID),
    (lambda p: setattr(p, "precision", 7), B.MECH_E_INVALID),
    (lambda p: setattr(p, "ab2_start", 3), B.MECH_E_INVALID),
    (lambda p: setattr(p, "flags", 0x100), B.MECH_E_INVALID),
    (lambda p: setattr(p, "voxel_size", 0.0), B.MECH_E_INVALID),
    (lambda p: setattr(p, "voxel_size", float("nan")), B.MECH_E_INVALID),
    (lambda p: setattr(p, "dt", -0.1), B.MECH_E_INVALID),
    (lambda p: setattr(p, "c_rep", float("inf")), B.MECH_E_INVALID),
    (lambda p: setattr(p, "rel_adh_distance", 0.5), B.MECH_E_INVALID),
    (lambda p: setattr(p, "n_types", 9), B.MECH_E_INVALID),
    (lambda p: setattr(p, "n_types", 0), B.MECH_E_INVALID),
    (lambda p: p.domain_hi.__setitem__(0, -200.0), B.MECH_E_INVALID),
    # the quantised prefilter needs |x| S < 2^52 (S = 256 per um at a 30 um voxel)
    (lambda p: p.domain_hi.__setitem__(1, 2.0 ** 45), B.MECH_E_INVALID),
    # ... and its threshold an int16: ceil(2^-20 |x| S) + 2 * 2^12 + 3 < 2^15, which fails
    # from |x| ~ 1.007e8 um at S = 256 (-t would wrap and drop pairs)
    (lambda p: p.domain_lo.__setitem__(2, -1.02e8), B.MECH_E_INVALID),
    (lambda p: p.domain_lo.__setitem__(2, -2.4e8), B.MECH_E_INVALID),
    (lambda p: p.domain_hi.__setitem__(0, 3.0e8), B.MECH_E_INVALID),
    (lambda p: setattr(p, "voxel_size", 1e-40), B.MECH_E_INVALID),
])
def test_workspace_bytes_rejects_bad_params(mutate, code):
    p, pop = _p()
    mutate(p)
    with pytest.raises(B.MechError) as e:
        B.population_workspace_bytes(p, 10)
    assert e.value.code == code
    assert B.mech_last_error() != ""


def test_asymmetric_adhesion_matrix_rejected():
    pop = workloads.spheroid(100, seed=3)
    p = B.params_of(pop)
    p.c_adh[1] = 0.2  # C[0][1] != C[1][0]
    with pytest.raises(B.MechError) as e:
        B.create_population(p, pop.pos, pop.radius, pop.type)
    assert e.value.code == B.MECH_E_INVALID and "symmetric" in B.mech_last_error()


@pytest.mark.parametrize("case,code", [
    ("nan_pos", B.MECH_E_INVALID), ("out_of_domain", B.MECH_E_OUT_OF_DOMAIN),
    ("bad_radius", B.MECH_E_INVALID), ("bad_type", B.MECH_E_INVALID),
    ("voxel_too_small", B.MECH_E_VOXEL_TOO_SMALL), ("nan_vprev", B.MECH_E_INVALID),
    ("length_mismatch", B.MECH_E_INVALID)])
def test_create_rejects_bad_cells_before_any_device_call(case, code):
    pop = workloads.plain(50, seed=4)
    p = B.params_of(pop)
    pos, rad, typ, vp = pop.pos.copy(), pop.radius.copy(), pop.type.copy(), None
    if case == "nan_pos":
        pos[3, 1] = np.nan
    elif case == "out_of_domain":
        pos[7, 2] = pop.hi[2] + 1e-9
    elif case == "bad_radius":
        rad[0] = -1.0
    elif case == "bad_type":
        typ[5] = 1
    elif case == "voxel_too_small":
        rad[9] = 12.5  # 1.25 * 2 * 12.5 = 31.25 > 30
    elif case == "nan_vprev":
        vp = np.zeros_like(pos)
        vp[2, 0] = np.inf
    elif case == "length_mismatch":
        rad = rad[:-1]
    with pytest.raises(B.MechError) as e:
        B.create_population(p, pos, rad, typ, vp)
    assert e.value.code == code, B.mech_last_error()


def test_prefilter_bound_accepts_large_valid_domains():
    """Just inside the threshold bound a domain is accepted (S = 256 per um at 30 um:
    ceil(2^-20 * 1.0e8 * 256) = 24,415 units, + 8192 + 3 < 32,768)."""
    p, _ = _p()
    p.domain_lo[2] = -1.0e8
    assert B.population_workspace_bytes(p, 10) > 0


def test_workspace_bytes_scales_with_cells():
    p, _ = _p()
    a = B.population_workspace_bytes(p, 1000)
    b = B.population_workspace_bytes(p, 2000)
    assert b > a > 0
    p32, _ = _p(precision=B.MECH_FP32_KAHAN)
    assert B.population_workspace_bytes(p32, 1000) > 0


def test_null_handles_are_rejected():
    lib = B.lib()
    assert lib.step_mechanics(None, 1) == B.MECH_E_INVALID
    assert lib.read_stats(None, None, None, None) == B.MECH_E_INVALID
    assert lib.read_xcd_split(None, None) == B.MECH_E_INVALID
    assert lib.destroy_population(None) == B.MECH_OK
    assert lib.population_stream(None) is None


def test_batch_capacity_validation():
    p = B.make_params((0, 0, 0), (1, 1, 1))
    assert B.batch_workspace_bytes(p, 1000, 500, 4) > B.batch_workspace_bytes(p, 100, 500, 4)
    for args in ((-1, 10, 1), (10, 0, 1), (10, 10, 0)):
        with pytest.raises(B.MechError):
            B.batch_workspace_bytes(p, *args)
    # voxels a request needs: ceil per axis, at least one
    assert B.batch_request_voxels(p, (-100, -100, -100), (100, 100, 100)) == 7 ** 3
    assert B.batch_request_voxels(p, (0, 0, 0), (90, 90, 0)) == 9
    with pytest.raises(B.MechError):
        B.batch_request_voxels(p, (0, 0, 0), (-1, 1, 1))


def test_population_workspace_is_a_one_slot_batch():
    pop = workloads.plain(1000)
    p = B.params_of(pop)
    v = B.batch_request_voxels(p, pop.lo, pop.hi)
    assert B.population_workspace_bytes(p, pop.n) == B.batch_workspace_bytes(p, pop.n, v, 1)


def test_serving_arena_fits_budget_and_limits():
    """The server sizes its arena from an HBM budget within the library's limits (no GPU
    needed: workspace sizes are computed on the host)."""
    from paper_2306_11544_amd.serve import capacity_for_budget
    p = B.make_params((0, 0, 0), (1, 1, 1), c_adh=workloads.C_ADH_2, precision=B.MECH_FP32)
    for budget in (4 << 20, 1 << 30, 200 << 30):
        cells, vox = capacity_for_budget(p, budget, 1.6, 1024)
        assert 0 < cells < 2 ** 31 and 0 < vox < 2 ** 30
        assert B.batch_workspace_bytes(p, cells, vox, 1024) <= budget


def test_binding_fails_loudly_without_the_library(monkeypatch, tmp_path):
    """No CPU fallback: with libmech.so missing the binding raises."""
    monkeypatch.setattr(B, "_lib", None)
    monkeypatch.setattr(B, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(ImportError):
        B.lib()


def test_profile_hash_ignores_comments_only():
    from paper_2306_11544_amd.rocprof_summary import code_of
    a = 'int f(int x) { return x + 1; } // one\n/* block */ const char* s = "a // b";\n'
    b = 'int f(int x)  {\n  return x + 1;\n}\n// two\nconst char* s = "a // b";'
    c = 'int f(int x) { return x + 2; }\nconst char* s = "a // b";'
    assert code_of(a) == code_of(b) != code_of(c)
    assert '"a // b"' in code_of(a)


def test_plain_c_client(tmp_path):
    """The boundary is a C ABI: a C program built against include/mech.h alone links
    libmech.so and gets the documented answers (no GPU needed for these calls)."""
    B.lib()  # builds nothing; fails loudly if the library is missing
    exe = tmp_path / "client"
    src = os.path.join(ROOT, "tests", "c_abi_client.c")
    subprocess.run(["gcc", "-std=c11", "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"), src,
                    B.LIB_PATH, f"-Wl,-rpath,{os.path.dirname(B.LIB_PATH)}", "-o", str(exe)],
                   check=True)
    res = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert res.returncode == 0, res.stdout + res.stderr
    assert "client ok" in res.stdout


def test_no_device_is_reported_as_a_device_error():
    """Without a GPU, creation fails with MECH_E_DEVICE and a message (no crash, no CPU
    fallback)."""
    if B.lib().mech_device_count() > 0:
        pytest.skip("a GPU is present")
    pop = workloads.plain(50, seed=4)
    with pytest.raises(B.MechError) as e:
        B.create_population(B.params_of(pop), pop.pos, pop.radius, pop.type)
    assert e.value.code == B.MECH_E_DEVICE
    assert "device" in B.mech_last_error().lower()
