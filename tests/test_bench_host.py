"""Host logic of bench.py, on the CPU: the frozen per-term operation counts
the roofline fractions are priced with (the method's work, independent of
how a kernel implements it), the roofline arithmetic, the tie between a
committed counter summary and the device sources it measured, and the
one-GPU contract."""
import os
import subprocess
import sys

import pytest

import bench


def test_frozen_counts_are_the_documented_sums():
    """Each count is the sum of the method's per-term steps as listed beside
    FLOPS (h = M S 15, six binary64 sines 96, exp 27, ...); a change of a
    kernel must not move them."""
    spots64 = 15 + 3 + 6 + 96 + 6 + 2
    spots_mixed = {"f64": 24, "f32": 60 + 6 + 1 + 4}
    gauss64 = 15 + 3 + 9 + 27 + 2
    adjoint64 = 15 + 15 + 3 + 9 + 27 + 2 + 39 + 1
    background64 = 3 + 5 + 1 + 1 + 3 + 1 + 23 + 3
    assert bench.FLOPS == {
        "spots": {"fp64": {"f64": spots64, "f32": 0}, "mixed": spots_mixed},
        "gauss_fwd": {"fp64": {"f64": gauss64, "f32": 0}, "mixed": {"f64": 28, "f32": 2 + 1 + 4}},
        "adjoint": {"fp64": {"f64": adjoint64, "f32": 0}, "mixed": {"f64": 43, "f32": 2 + 2 + 39 + 1}},
        "background": {"fp64": {"f64": background64, "f32": 0}, "mixed": {"f64": 0, "f32": background64 + 3}},
    }
    assert (spots64, gauss64, adjoint64, background64) == (128, 56, 111, 40)


def test_roofline_arithmetic():
    """MI355X vector peaks from the unit counts and clock (78.6 / 157.3
    TFLOP/s); a binary64 path at exactly its peak rate has frac 1; a mixed
    term is priced at both peaks."""
    assert bench.PEAK["f64"] == pytest.approx(78.6432e12)
    assert bench.PEAK["f32"] == pytest.approx(157.2864e12)
    f = bench.FLOPS["spots"]["fp64"]
    at_peak = bench.PEAK["f64"] / 128
    r = bench.roofline_of(f, at_peak)
    assert r["frac"] == pytest.approx(1.0) and r["achieved"] == pytest.approx(78.6432)
    r = bench.roofline_of(f, 0.5 * at_peak)
    assert r["frac"] == pytest.approx(0.5) and r["peak"] == pytest.approx(78.6432)
    m = bench.FLOPS["spots"]["mixed"]
    t_term = 24 / bench.PEAK["f64"] + 71 / bench.PEAK["f32"]
    r = bench.roofline_of(m, 1e11)
    assert r["frac"] == pytest.approx(1e11 * t_term)
    assert r["achieved"] == pytest.approx(95 * 1e11 / 1e12)
    assert r["peak"] == pytest.approx(95 / t_term / 1e12)


def test_profile_keys_follow_the_device_sources(monkeypatch):
    """A committed summary's figures are used only while the device sources
    are the ones its counters measured (the sha it records), never for a
    missing file."""
    names = [n for n in os.listdir(os.path.join(bench.HERE, "profiles")) if n.endswith("_counters.txt")]
    assert names
    for name in names:
        with open(os.path.join(bench.HERE, "profiles", name)) as fp:
            line = next(l for l in fp if l.startswith("# bench-keys "))
        sha = bench.json.loads(line[len("# bench-keys "):])["kernel_src_sha"]
        monkeypatch.setattr(bench, "kernel_src_sha", lambda: sha)
        keys = bench.profile_keys(name)
        assert keys is not None and keys["source"] == f"profiles/{name}"
        monkeypatch.setattr(bench, "kernel_src_sha", lambda: "0" * 16)
        assert bench.profile_keys(name) is None
    assert bench.profile_keys("no_such_summary.txt") is None


def test_more_than_one_gpu_is_refused():
    """--gpus N > 1 exits with status 2 and says why, before touching a GPU."""
    r = subprocess.run([sys.executable, os.path.join(bench.HERE, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr and r.stdout == ""
