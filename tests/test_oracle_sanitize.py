"""The oracle under host sanitizers: oracle/sanitize_driver.cpp calls every
oracle entry point (including the empty cases) and is built with
AddressSanitizer and UndefinedBehaviorSanitizer (g++, host code only), then run
as its own executable; any invalid access or undefined arithmetic fails it."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = [os.path.join(ROOT, "oracle", f) for f in
       ("sanitize_driver.cpp", "rogs_oracle.cpp", "rogs_oracle_grid.cpp")]


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_oracle_runs_clean_under_asan_and_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_sanitize")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fopenmp",
           "-ffp-contract=off", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           *SRC, "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True, timeout=300)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:halt_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1", OMP_NUM_THREADS="2")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert "oracle sanitizer run: ok" in r.stdout
