"""The serving runtime under host sanitizers: tests/serve_sanitize_driver.cpp,
linked with the library sources whose host code is built with AddressSanitizer
and UndefinedBehaviorSanitizer (device code unchanged), runs a server over a
small map with requests from two threads, the argument errors, the
statistics and shutdown; any invalid host access or undefined arithmetic in
the runtime fails it.  Leak detection is off: the HIP runtime keeps
allocations until the process ends."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
EXE = os.path.join(ROOT, "tests", "_bin", "serve_sanitize")

pytestmark = pytest.mark.gpu


def test_serve_runtime_runs_clean_under_asan_and_ubsan():
    assert os.path.exists(EXE), "build the driver first (paper_2405_14342_amd/build.py)"
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:protect_shadow_gap=0:halt_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([EXE], capture_output=True, text=True, timeout=120, env=env)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert "serve sanitizer run: ok" in r.stdout
