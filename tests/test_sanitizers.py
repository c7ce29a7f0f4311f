"""AddressSanitizer and UndefinedBehaviorSanitizer on the CPU side (no GPU needed).

1. The two oracles, built with gcc -fsanitize=address,undefined together with a plain C
   driver (sanitize_oracle_main.c) that calls every oracle function on small, ragged and
   degenerate inputs.
2. The host side of libmech.so (parameter and domain validation, arena layout, budget
   sizing, the microenvironment's validation and elimination set-up, the
   allocation-free call's checks), built by hipcc with the sanitizers on the host pass
   only (-Xarch_host before each -fsanitize=; device code is not instrumented), and
   driven by the plain C ABI client built with the same compiler's sanitizers.

A sanitizer report makes the program exit non-zero (-fno-sanitize-recover=all).
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN_ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1", OMP_NUM_THREADS="2")

pytestmark = pytest.mark.slow


def _run(cmd, **kw):
    res = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert res.returncode == 0, (" ".join(cmd), res.stdout[-3000:], res.stderr[-3000:])
    return res


def test_oracles_under_asan_and_ubsan(tmp_path):
    exe = str(tmp_path / "san_oracle")
    _run(["gcc", "-std=c11", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
          "-fno-omit-frame-pointer", "-ffp-contract=off", "-fopenmp",
          os.path.join(ROOT, "tests", "sanitize_oracle_main.c"),
          os.path.join(ROOT, "oracle", "mech_oracle.c"),
          os.path.join(ROOT, "oracle", "diffusion_oracle.c"), "-o", exe, "-lm"])
    res = _run([exe], env=SAN_ENV, timeout=300)
    assert "oracle sanitized ok" in res.stdout


def test_library_host_code_under_asan_and_ubsan(tmp_path):
    from paper_2306_11544_amd import build as hip_build
    clang = "/opt/rocm/llvm/bin/clang"
    if not os.path.exists(clang):
        clang = shutil.which("clang")
    assert clang, "clang (the ROCm LLVM) is needed to link against the sanitized library"
    lib = str(tmp_path / "libmech_san.so")
    san = []
    for flag in ("-fsanitize=address", "-fsanitize=undefined", "-fno-sanitize-recover=all",
                 "-fno-omit-frame-pointer"):
        san += ["-Xarch_host", flag]
    flags = [f for f in hip_build.HIP_FLAGS if f != "-O3"]
    _run([hip_build.hipcc(), *flags, "-O1", "-g", *san, "-I", hip_build.INCLUDE, *hip_build.SOURCES,
          "-o", lib], timeout=900)
    exe = str(tmp_path / "client_san")
    _run([clang, "-std=c11", "-Wall", "-Werror", "-g", "-fsanitize=address,undefined",
          "-fno-sanitize-recover=all", "-I", os.path.join(ROOT, "include"),
          os.path.join(ROOT, "tests", "c_abi_client.c"), lib, f"-Wl,-rpath,{tmp_path}", "-o", exe])
    res = _run([exe], env=SAN_ENV, timeout=300)
    assert "client ok" in res.stdout
