"""The C ABI's host code under AddressSanitizer and UndefinedBehaviorSanitizer.

The CPU tests of the ABI (tests/test_abi_cpu.py: argument validation,
workspace sizing, the batched and static entry points' checks) run against
_build_san/libmf_san.so, whose host code carries ASan and UBSan checks, in a
Python process with the sanitizer runtime preloaded.  Any sanitizer report
fails the run (UBSan does not recover; ASan aborts on its first error).
Leak detection is off: the interpreter itself is not instrumented.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
from paper_1511_06103_amd import build  # noqa: E402

RUNNER = """
import sys
sys.path.insert(0, {root!r})
from paper_1511_06103_amd import mf
mf.LIB_PATH = {lib!r}
import pytest
sys.exit(pytest.main(['-q', '-p', 'no:cacheprovider', {tests!r}]))
"""


def test_abi_tests_pass_under_asan_and_ubsan():
    rt = build.sanitizer_runtime()
    if rt is None:
        pytest.skip("no clang AddressSanitizer runtime in this ROCm install")
    if not os.path.exists(build.LIB_SAN):
        build.build(sanitize=True)
    syms = subprocess.run(["nm", "-D", "--undefined-only", build.LIB_SAN], capture_output=True, text=True).stdout
    assert "__asan_report_load" in syms and "__ubsan_handle" in syms, "host code is not instrumented"
    env = dict(os.environ, LD_PRELOAD=rt, ASAN_OPTIONS="detect_leaks=0:halt_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    code = RUNNER.format(root=ROOT, lib=build.LIB_SAN, tests=os.path.join(ROOT, "tests", "test_abi_cpu.py"))
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=env, cwd="/tmp", timeout=600)
    out = r.stdout + r.stderr
    assert "AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
    assert r.returncode == 0 and " passed" in out, out[-4000:]
