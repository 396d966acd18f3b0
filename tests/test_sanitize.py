"""The CPU oracle and the library's host code under AddressSanitizer and
UndefinedBehaviorSanitizer.

Each is built into a temporary directory with the sanitizers on (the oracle
with gcc; the library's host code with hipcc's host pass, its device code as
usual) and the CPU tests that exercise it run again in a child process with
the matching runtime preloaded.  Any out-of-bounds access, use after free or
undefined behaviour aborts the child and fails here.  Leak checking is off:
the Python interpreter itself keeps allocations alive at exit.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORACLE_TESTS = ["test_oracle_core.py", "test_oracle_inert.py", "test_oracle_init_stats.py", "test_oracle_field.py",
                "test_oracle_pair.py", "test_oracle_nfold.py", "test_oracle_mcp_mlp.py", "test_oracle_mcp_pins.py",
                "test_oracle_markov.py"]
LIBRARY_TESTS = ["test_abi.py", "test_table.py", "wip_no_alloc.py", "test_zz_no_alloc.py"]


def _run(env_extra, tests, tmp):
    env = dict(os.environ)
    env.update(env_extra)
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1:halt_on_error=1"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    files = [os.path.join(ROOT, "tests", t) for t in tests if os.path.exists(os.path.join(ROOT, "tests", t))]
    cmd = [sys.executable, "-m", "pytest", "-q", "-x", "-m", "not gpu and not slow", "-p", "no:cacheprovider",
           "--rootdir", ROOT] + files
    r = subprocess.run(cmd, cwd=tmp, env=env, capture_output=True, text=True, timeout=900)
    out = r.stdout + r.stderr
    assert "ERROR: AddressSanitizer" not in out, out[-4000:]
    assert "runtime error:" not in out, out[-4000:]
    assert r.returncode == 0, out[-4000:]
    return out


def test_oracle_under_sanitizers(tmp_path):
    from oracle import build as oracle_build

    lib = oracle_build.build(sanitize=True, out=str(tmp_path / "liboracle_san.so"))
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    ubsan = subprocess.run(["gcc", "-print-file-name=libubsan.so"], capture_output=True, text=True).stdout.strip()
    if not os.path.isabs(asan) or not os.path.exists(asan):
        pytest.skip("gcc's AddressSanitizer runtime is not installed")
    out = _run({"LD_PRELOAD": f"{asan}:{ubsan}", "ORACLE_LIB": lib}, ORACLE_TESTS, str(tmp_path))
    assert " passed" in out


def test_library_host_code_under_sanitizers(tmp_path):
    from paper_1007_3509_amd import _build as hip_build

    clang_rt = None
    base = "/opt/rocm/llvm/lib/clang"
    if os.path.isdir(base):
        for v in sorted(os.listdir(base)):
            p = os.path.join(base, v, "lib", "linux", "libclang_rt.asan-x86_64.so")
            if os.path.exists(p):
                clang_rt = p
    if clang_rt is None or not os.path.exists(hip_build.HIPCC):
        pytest.skip("hipcc or clang's AddressSanitizer runtime is not installed")
    lib = hip_build.build(sanitize_host=True, out=str(tmp_path / "libhmc_san.so"))
    out = _run({"LD_PRELOAD": clang_rt, "HMC_LIBRARY": lib}, LIBRARY_TESTS, str(tmp_path))
    assert " passed" in out
