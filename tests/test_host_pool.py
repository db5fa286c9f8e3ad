"""The plan builder's host loops (persistent worker pool) under ThreadSanitizer.

tests/host_pool_test.cpp is built with g++ -fsanitize=thread against
paper_2607_19489_amd/csrc/host_pool.h alone (no HIP, no GPU) and run: ranges,
nested loops, exception order, concurrent callers; any race report fails.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
OUT = os.path.join(ROOT, "paper_2607_19489_amd", "_build", "sanitize")


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_host_pool_under_tsan():
    os.makedirs(OUT, exist_ok=True)
    exe = os.path.join(OUT, "host_pool_test_tsan")
    subprocess.run(["g++", "-std=c++17", "-O1", "-g", "-fsanitize=thread", "-pthread",
                    "-I", os.path.join(ROOT, "paper_2607_19489_amd", "csrc"),
                    os.path.join(ROOT, "tests", "host_pool_test.cpp"), "-o", exe], check=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300,
                       env=dict(os.environ, TSAN_OPTIONS="halt_on_error=1"))
    assert r.returncode == 0 and "ok" in r.stdout, r.stdout[-2000:] + r.stderr[-4000:]
    assert "WARNING: ThreadSanitizer" not in r.stderr, r.stderr[-4000:]
