"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer, CPU
only.  The C ABI tests (``test_abi.py``: exports, struct layout, argument
validation before any device work, error strings) run against a build whose
host code in ``runtime.hip`` carries both sanitizers (validation never
reaches the GPU), and the C++ oracle's tests run against a sanitized build
of the oracle.  A sanitizer report (heap overflow, use after free, signed
overflow, a bad shift or cast, ...) aborts the child process, which fails
the test."""

import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _assert_instrumented(lib):
    """The library under test really calls into both sanitizer runtimes."""
    syms = subprocess.check_output(["nm", "-D", lib], text=True)
    assert "__asan_report" in syms and "__ubsan_handle" in syms, lib


def test_abi_suite_under_asan_and_ubsan():
    from paper_2001_11806_amd import build_sanitized as S
    try:
        lib = S.build()
        rt = S.asan_runtime()
    except (RuntimeError, subprocess.CalledProcessError) as e:
        pytest.fail("sanitizer build failed: %s" % e)
    _assert_instrumented(lib)
    env = dict(os.environ, LD_PRELOAD=rt, LBM_MI355X_LIB=lib,
               # CPython's own allocations are never freed at exit: leak
               # checking would only report the interpreter
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    res = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider",
                          os.path.join(ROOT, "tests", "test_abi.py")],
                         cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    out = res.stdout + res.stderr
    print(out[-3000:])
    assert res.returncode == 0, out[-3000:]
    assert "ERROR: AddressSanitizer" not in out and "runtime error:" not in out
    assert " passed" in out


def test_cpp_oracle_under_asan_and_ubsan():
    """The C++ oracle's equality with the numpy oracle (every stencil x
    method, FP64 and emulated FP16 storage, walls, forces) and its MRT basis
    pins, run against the oracle built with -fsanitize=address,undefined."""
    from oracle import cpu
    try:
        lib = cpu.build_sanitized()
    except subprocess.CalledProcessError as e:
        pytest.fail("sanitized oracle build failed: %s" % e)
    _assert_instrumented(lib)
    rt = subprocess.check_output(["gcc", "-print-file-name=libasan.so"], text=True).strip()
    env = dict(os.environ, LD_PRELOAD=rt, LBM_ORACLE_LIB=lib,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    res = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider",
                          os.path.join(ROOT, "tests", "test_oracle_cpp.py"),
                          "-k", "(equals_numpy and (f64 or f16)) or mrt_basis or even_odd"],
                         cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    out = res.stdout + res.stderr
    print(out[-3000:])
    assert res.returncode == 0, out[-3000:]
    assert "ERROR: AddressSanitizer" not in out and "runtime error:" not in out
    assert " passed" in out
