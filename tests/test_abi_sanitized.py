"""The host runtime under AddressSanitizer and UndefinedBehaviorSanitizer (CPU
only): the library is rebuilt with api.hip's host code instrumented, and the
cases of tests/abi_host_cases.py run in a child process with the sanitizer
runtime preloaded.  Any report (an invalid memory access, signed overflow,
invalid shift, misaligned or null access) fails the test."""
import os
import shutil
import subprocess
import sys

import pytest

from paper_2606_21125_amd import build

HERE = os.path.dirname(os.path.abspath(__file__))


def test_host_runtime_under_sanitizers():
    if not os.path.exists(build.HIPCC) and not shutil.which("hipcc"):
        pytest.skip("hipcc not available")
    rt = build.asan_runtime()
    if not rt:
        pytest.skip("no shared AddressSanitizer runtime")
    lib = build.build_host_sanitized()
    env = dict(os.environ)
    env["LD_PRELOAD"] = rt
    env["ASAN_OPTIONS"] = "detect_leaks=0:halt_on_error=1:abort_on_error=0"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    res = subprocess.run([sys.executable, os.path.join(HERE, "abi_host_cases.py"), lib],
                         env=env, capture_output=True, text=True, timeout=600)
    report = res.stdout[-3000:] + res.stderr[-6000:]
    assert res.returncode == 0, report
    assert "runtime error" not in res.stderr, report
    assert "AddressSanitizer" not in res.stderr, report
    assert "statuses seen" in res.stdout
