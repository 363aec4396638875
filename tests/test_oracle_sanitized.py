"""The oracle's pins, run against an AddressSanitizer + UndefinedBehavior-
Sanitizer build of oracle.c (every report fatal).  Out-of-bounds ghost or
pencil accesses, use of freed scratch, signed overflow in index arithmetic
or misaligned loads in the oracle abort the run.  CPU only."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_oracle_pins_pass_under_asan_and_ubsan(tmp_path):
    from oracle.build import asan_runtime, build
    lib = build(force=True, lib=str(tmp_path / "liboracle_asan.so"), sanitize=True)
    env = dict(os.environ, HYDRO_ORACLE_LIB=lib, LD_PRELOAD=asan_runtime(),
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1",
               OMP_NUM_THREADS="2")
    cmd = [sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
           "-m", "not slow", os.path.join(ROOT, "tests", "test_oracle_pins.py"),
           os.path.join(ROOT, "tests", "test_amr_step_pins.py")]
    r = subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
    assert "ERROR: AddressSanitizer" not in r.stderr
    assert "runtime error" not in r.stderr
