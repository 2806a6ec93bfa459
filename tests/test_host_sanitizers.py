"""The C ABI tests (``test_abi.py``: exports, struct layout, argument
validation before any device work, error strings) run against a build whose
host code in ``runtime.hip`` carries AddressSanitizer and
UndefinedBehaviorSanitizer.  CPU only: validation never reaches the GPU.
A sanitizer report (heap overflow, use after free, signed overflow, a bad
shift or cast, ...) aborts the child process, which fails this test."""

import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_abi_suite_under_asan_and_ubsan():
    from paper_2001_11806_amd import build_sanitized as S
    try:
        lib = S.build()
        rt = S.asan_runtime()
    except (RuntimeError, subprocess.CalledProcessError) as e:
        pytest.fail("sanitizer build failed: %s" % e)
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
