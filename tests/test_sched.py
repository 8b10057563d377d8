"""The shot server's scheduling logic (paper_2205_07976_amd/csrc/xrt_sched.h:
arena allocation, admission in arrival order by HBM footprint and resident
slots, chunking, publication by least published work, compute then reduce
phases of split shots, ring sequence numbers) on the CPU against a simulated
device.  The checks are in sched_check.cpp beside this file; this test builds
it with the host compiler and runs it."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


def test_scheduler_checks(tmp_path):
    cxx = shutil.which("g++") or shutil.which("c++")
    if cxx is None:
        pytest.skip("no host C++ compiler")
    exe = tmp_path / "sched_check"
    subprocess.run([cxx, "-std=c++17", "-O1", "-Wall", "-Wextra", "-Werror", "-o", str(exe),
                    os.path.join(HERE, "sched_check.cpp")], check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300)
    print(r.stdout)
    assert r.returncode == 0, r.stderr
    assert "all scheduler checks passed" in r.stdout
