"""The host-side ABI tests (tests/test_abi.py) against a build of the library
whose host code runs under AddressSanitizer and UndefinedBehaviorSanitizer
(CPU only: argument validation, plan sizes, the host Bessel series; any report
aborts the child process)."""

import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_abi_under_host_sanitizers():
    from paper_2403_04351_amd import build_sanitized as bs

    lib = bs.build()
    env = dict(os.environ, LTD_LIBRARY=lib, LD_PRELOAD=bs.asan_runtime(),
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_abi.py")], cwd=ROOT, env=env, capture_output=True,
                       text=True, timeout=600)
    print(r.stdout[-2000:], r.stderr[-4000:])
    assert r.returncode == 0
    assert "passed" in r.stdout and "AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr
