"""The CPU oracle built with AddressSanitizer and UndefinedBehaviorSanitizer
(g++, -fno-sanitize-recover) and run through every entry point on small 2D
and 3D cavities by tests/oracle_sanitize_driver.cpp: no out-of-bounds
access, use after free, leak or undefined operation (test infrastructure
checks of the oracle itself; no GPU)."""
import os
import shutil
import subprocess
import tempfile

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_oracle_under_address_and_undefined_behaviour_sanitizers():
    with tempfile.TemporaryDirectory() as tmp:
        exe = os.path.join(tmp, "oracle_sanitize")
        cmd = ["g++", "-std=c++17", "-O1", "-g", "-fopenmp", "-ffp-contract=off",
               "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
               "-fno-omit-frame-pointer", os.path.join(HERE, "oracle_sanitize_driver.cpp"),
               "-o", exe]
        subprocess.run(cmd, check=True, capture_output=True, text=True, timeout=600)
        env = dict(os.environ, OMP_NUM_THREADS="2",
                   ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
                   UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
        r = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env)
        assert r.returncode == 0, r.stdout[-4000:] + r.stderr[-4000:]
        assert "sanitizer driver ok" in r.stdout
