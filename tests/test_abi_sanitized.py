"""The C ABI's argument checks under AddressSanitizer and
UndefinedBehaviorSanitizer (host code), on the CPU: tests/abi_check.cpp calls
every entry point with NULL handles, NULL pointers and out-of-range sizes and
checks the documented status codes; the sanitizers abort on a memory error or
undefined behaviour. Where a GPU is present the same driver also walks a real
plan's state errors."""
import os
import subprocess

import pytest


@pytest.mark.slow
def test_abi_under_sanitizers():
    from paper_1706_08575_amd import build as B
    exe = B.build_abi_check()
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    out = r.stdout + r.stderr
    assert "AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
    assert r.returncode == 0, out[-4000:]
    assert "abi_check: 0 failure(s)" in out
