"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer: the library's host side
(api.cpp, plan.cpp, coeffs.cpp and the launch wrappers) built with both sanitizers, running the
host-only ABI checks (tests/test_abi.py: exported symbols, configuration validation, footprints,
every coupling table against the oracle's) on the CPU.  Any sanitizer report fails the run."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_abi_checks_pass_under_asan_and_ubsan():
    from paper_2102_08384_amd import build
    if not os.path.exists(build.HIPCC):
        pytest.skip("hipcc not available")
    lib = build.build_sanitized()
    env = dict(os.environ)
    env.update({"LD_PRELOAD": build.sanitizer_runtime(), "PW_LIB": lib,
                # python itself is not instrumented: its allocations are not leaks of ours
                "ASAN_OPTIONS": "detect_leaks=0:halt_on_error=1:abort_on_error=0",
                "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"})
    r = subprocess.run([sys.executable, "-m", "pytest", os.path.join(ROOT, "tests", "test_abi.py"), "-q",
                        "-p", "no:cacheprovider"], cwd=ROOT, env=env, capture_output=True, text=True,
                       timeout=900)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "ERROR: AddressSanitizer" not in out and "runtime error:" not in out, out[-4000:]
    assert " passed" in out
