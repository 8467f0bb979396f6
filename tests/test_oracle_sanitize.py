"""The CPU oracle built with AddressSanitizer and UndefinedBehaviorSanitizer (g++, host code only)
and run over every entry point and edge case (tests/oracle_sanitize_driver.cpp): no memory error,
no undefined behaviour."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_oracle_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_sanitize")
    src = os.path.join(HERE, "oracle_sanitize_driver.cpp")
    build = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fopenmp",
             "-ffp-contract=off", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
             src, "-o", exe]
    subprocess.run(build, check=True, capture_output=True, text=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1", OMP_NUM_THREADS="2")
    res = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert res.returncode == 0, res.stderr[-4000:]
    assert "runtime error" not in res.stderr and "AddressSanitizer" not in res.stderr, res.stderr[-4000:]
    assert "oracle sanitizer run: ok" in res.stdout
