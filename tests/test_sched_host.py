"""Host bookkeeping of the serving loop (admission, sequence rules, the
stream timeline, invalid spans, latency percentiles), compiled with g++ from
the library's device-free source and driven by a fake executor on the CPU
(tests/cpp/test_sched.cpp)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1509_00186_amd", "csrc")


@pytest.mark.skipif(shutil.which("g++") is None, reason="no g++")
def test_serving_bookkeeping_with_fake_executor(tmp_path):
    exe = str(tmp_path / "test_sched")
    subprocess.run(["g++", "-std=c++17", "-O1", "-Wall", "-I", CSRC,
                    os.path.join(ROOT, "tests", "cpp", "test_sched.cpp"),
                    os.path.join(CSRC, "cdd_sched.cpp"), "-o", exe], check=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    print(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "all passed" in r.stdout
