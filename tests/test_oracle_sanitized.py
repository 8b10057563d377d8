"""The oracle (oracle/xro.c) under AddressSanitizer and
UndefinedBehaviorSanitizer: tests/oracle_check.c drives every entry point on
small shots that reach every branch (sub-pixels, layers, off-axis sources,
spindle steps, domains, table misses, both shapes, the gradient, the
background and every branch of its curve)."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def test_oracle_under_sanitizers(tmp_path):
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no host C compiler")
    probe = subprocess.run([cc, "-fsanitize=address,undefined", "-x", "c", "-", "-o", str(tmp_path / "probe")],
                           input="int main(void) { return 0; }\n", capture_output=True, text=True)
    if probe.returncode:
        pytest.skip("host compiler without sanitizer runtimes")
    exe = tmp_path / "oracle_check"
    subprocess.run([cc, "-std=c11", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                    "-fno-omit-frame-pointer", "-ffp-contract=off", "-fopenmp", "-Wall", "-Werror",
                    "-o", str(exe), os.path.join(HERE, "oracle_check.c"), os.path.join(ROOT, "oracle", "xro.c"),
                    "-lm"], check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-3000:]
    assert "oracle checks passed" in r.stdout
