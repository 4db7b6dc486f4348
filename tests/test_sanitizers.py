"""The oracle and the host side of the C ABI built with AddressSanitizer and
UndefinedBehaviorSanitizer (CPU only).

* The oracle (plain C) is compiled with -fsanitize=address,undefined into a
  separate shared library, and a subset of its pins runs against that build in
  a child Python process (the sanitizer runtime preloaded, leak checking off
  for the interpreter's own allocations): out-of-bounds accesses, use after
  free and undefined arithmetic in the oracle fail the run.
* The host-side ABI code (argument validation, 1-D rules and tables, element
  dimensions, block layouts, the concatenated index, the axis-order planner)
  is compiled with clang and both sanitizers into a driver executable whose
  kernel launchers are stubs that abort: every invalid call must be rejected
  before any launcher or HIP allocation is reached.
"""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CLANG = "/opt/rocm/llvm/bin/clang++"


def _gcc_runtime(name):
    out = subprocess.run(["gcc", "-print-file-name=" + name], stdout=subprocess.PIPE, text=True).stdout.strip()
    return out if os.path.isabs(out) and os.path.exists(out) else None


@pytest.fixture(scope="module")
def workdir(tmp_path_factory):
    return tmp_path_factory.mktemp("sanitize")


def test_oracle_pins_under_asan_ubsan(workdir):
    asan = _gcc_runtime("libasan.so")
    if shutil.which("gcc") is None or asan is None:
        pytest.skip("gcc with AddressSanitizer is not available")
    lib = str(workdir / "liborc_asan.so")
    subprocess.check_call(["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                           "-fno-sanitize-recover=undefined", "-ffp-contract=off", "-fopenmp", "-shared", "-fPIC",
                           "-std=c11", "-o", lib, os.path.join(ROOT, "oracle", "sf_oracle.c"), "-lm"])
    env = dict(os.environ)
    env.update({"SF_ORACLE_LIB": lib, "LD_PRELOAD": asan, "OMP_NUM_THREADS": "2",
                "ASAN_OPTIONS": "detect_leaks=0:abort_on_error=1",
                "UBSAN_OPTIONS": "print_stacktrace=1:halt_on_error=1"})
    tests = ["tests/test_golden.py", "tests/test_oracle_vq.py",
             "tests/test_oracle_pins.py::test_closed_form_rules",
             "tests/test_oracle_pins.py::test_q1_unit_cube_closed_form",
             "tests/test_oracle_pins.py::test_box_equals_kronecker",
             "tests/test_oracle_pins.py::test_symmetry",
             "tests/test_oracle_pins.py::test_nce_curlcurl_kills_gradients",
             "tests/test_oracle_pins.py::test_dofmap_brute_force_matches_lattice_closed_form",
             "tests/test_oracle_pins.py::test_action_equals_matrix_times_u",
             "tests/test_oracle_svk.py::test_residual_is_energy_derivative_and_jacobian_is_residual_derivative"]
    tests = [t for t in tests if os.path.exists(os.path.join(ROOT, t.split("::")[0]))]
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", "-m", "not gpu"] + tests,
                       cwd=ROOT, env=env, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True, timeout=900)
    assert r.returncode == 0, r.stdout[-4000:]
    assert "ERROR: AddressSanitizer" not in r.stdout and "runtime error" not in r.stdout, r.stdout[-4000:]


def test_abi_host_code_under_asan_ubsan(workdir):
    if not os.path.exists(CLANG):
        pytest.skip("clang++ not available")
    exe = str(workdir / "abi_host_driver")
    csrc = os.path.join(ROOT, "paper_1711_02473_amd", "csrc")
    cmd = [CLANG, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
           "-I" + os.path.join(ROOT, "include"), "-o", exe,
           os.path.join(ROOT, "tests", "sanitize", "abi_host_driver.cpp"),
           os.path.join(csrc, "api.cpp"), os.path.join(csrc, "tables.cpp"),
           "-L/opt/rocm/lib", "-Wl,-rpath,/opt/rocm/lib", "-lamdhip64"]
    subprocess.check_call(cmd)
    env = dict(os.environ)
    env.update({"ASAN_OPTIONS": "detect_leaks=0:abort_on_error=1", "UBSAN_OPTIONS": "print_stacktrace=1"})
    r = subprocess.run([exe], env=env, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True, timeout=300)
    assert r.returncode == 0, r.stdout[-4000:]
    assert "abi host checks ok" in r.stdout
