"""The host C++ of the library (host_math.cpp: elliptic functions, Zolotarev coefficients,
tridiagonal eigensolvers, SplitMix64, colourings) built with g++ under the address and
undefined-behaviour sanitizers and run on its own checks (tests/host/host_math_check.cpp)."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_host_math_under_sanitizers(tmp_path):
    exe = str(tmp_path / "host_math_check")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           os.path.join(HERE, "host", "host_math_check.cpp"),
           os.path.join(ROOT, "paper_1901_02211_amd", "csrc", "host_math.cpp"), "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True, timeout=300)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0", UBSAN_OPTIONS="print_stacktrace=1")
    out = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert out.returncode == 0, out.stdout + out.stderr
    assert "0 failures" in out.stdout
