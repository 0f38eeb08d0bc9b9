"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer.

tests/sanitize/build_sanitized.py builds the library with the host pass of
every translation unit instrumented (device code as usual) and a C driver
that calls the C-ABI; the driver fails on any broken check and a sanitizer
report aborts it.  Host-only paths run here; the whole boundary on a GPU.
"""
import os
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "sanitize"))
import build_sanitized  # noqa: E402


def _exe():
    if not (os.path.exists(build_sanitized.EXE) and os.path.exists(build_sanitized.LIB)):
        build_sanitized.build()
    return build_sanitized.EXE


def _run(mode, leaks):
    env = dict(os.environ)
    env["ASAN_OPTIONS"] = f"detect_leaks={int(leaks)}:abort_on_error=1:halt_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    print(f"host_exercise {mode}", flush=True)
    r = subprocess.run([_exe(), mode], capture_output=True, text=True, env=env, timeout=240)
    report = r.stdout + r.stderr
    assert "AddressSanitizer" not in report and "runtime error" not in report, report[-4000:]
    assert r.returncode == 0 and f"host_exercise {mode}: ok" in r.stdout, report[-4000:]


def test_host_paths_clean_under_asan_ubsan():
    """Admission simulation over random streams and every entry point's argument checks."""
    _run("cpu", leaks=True)


@pytest.mark.gpu
def test_whole_boundary_clean_under_asan_ubsan():
    """Encode, prepare, MTTKRP (three forms), CP-ALS, batched, allocator hook, plan change,
    autotuner and server on device 0, with the host code instrumented (leak checks off:
    the HIP runtime keeps allocations until exit)."""
    _run("gpu", leaks=False)
