"""The FP64 oracle built with the address and undefined-behaviour sanitizers
(g++, host code only) and driven through every entry on small seeded cases
by tests/oracle_sanitize_main.cpp: no out-of-bounds access, use after free,
leak, signed overflow, misaligned or null access anywhere in the oracle."""
import os
import shutil
import subprocess
import tempfile

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_oracle_under_address_and_undefined_behaviour_sanitizers():
    with tempfile.TemporaryDirectory(prefix="orc_san_") as d:
        exe = os.path.join(d, "orc_san")
        cmd = ["g++", "-std=c++17", "-O1", "-g", "-fopenmp", "-ffp-contract=off",
               "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
               "-fno-sanitize-recover=all", "-o", exe,
               os.path.join(HERE, "oracle_sanitize_main.cpp")]
        subprocess.run(cmd, check=True, capture_output=True, text=True, timeout=600)
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
                   UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1", OMP_NUM_THREADS="2")
        r = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env)
        assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
        assert r.stdout.strip().endswith("ok"), r.stdout[-2000:]
        assert "runtime error" not in r.stderr, r.stderr[-4000:]
