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


def _build_and_run(cxx, tmp_path, name, flags):
    exe = tmp_path / name
    subprocess.run([cxx, "-std=c++17", "-Wall", "-Wextra", "-Werror", *flags, "-o", str(exe),
                    os.path.join(HERE, "sched_check.cpp")], check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300)
    print(r.stdout)
    assert r.returncode == 0, r.stderr
    assert "all scheduler checks passed" in r.stdout


def test_scheduler_checks(tmp_path):
    cxx = shutil.which("g++") or shutil.which("c++")
    if cxx is None:
        pytest.skip("no host C++ compiler")
    _build_and_run(cxx, tmp_path, "sched_check", ["-O1"])


def test_scheduler_checks_sanitized(tmp_path):
    """The same checks under AddressSanitizer and UndefinedBehaviorSanitizer
    (host code only): out-of-bounds access, use after free, leaks, signed
    overflow and the like in the scheduling logic fail the run."""
    cxx = shutil.which("g++") or shutil.which("c++")
    if cxx is None:
        pytest.skip("no host C++ compiler")
    probe = subprocess.run([cxx, "-fsanitize=address,undefined", "-x", "c++", "-", "-o", str(tmp_path / "probe")],
                           input="int main() { return 0; }\n", capture_output=True, text=True)
    if probe.returncode:
        pytest.skip("host compiler without sanitizer runtimes")
    _build_and_run(cxx, tmp_path, "sched_check_asan",
                   ["-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"])
