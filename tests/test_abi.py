"""The C-ABI library without a GPU: it loads, exports every entry point the
header declares, and its host-side paths (validation, cell matrices) behave
as documented.  No compute call is made."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import synth
from oracle import oracle as o
from paper_2205_07976_amd import xrt

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    txt = open(os.path.join(ROOT, "include", "xrt.h")).read()
    return sorted(set(re.findall(r"^\s*(?:xrt_status|const char \*)\s*(xrt_\w+)\s*\(", txt, re.M)))


def test_header_symbols_exported():
    lib = xrt.load()
    names = declared_symbols()
    assert len(names) >= 7
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(xrt.SYMBOLS)


def test_version():
    assert xrt.version() == (1, 0)


@pytest.mark.parametrize("make", [synth.tiny_shot, synth.micro_shot, lambda: synth.full_shot()])
def test_cell_mats_bitwise_equal_oracle(make):
    """The library builds the lab-frame cell matrices with the same operation
    sequence as the oracle: every bit agrees (this is what lets h agree)."""
    shot = make()
    assert np.array_equal(xrt.cell_mats(shot), o.cell_mats(shot))


def test_cell_mats_phi_steps():
    shot = synth.micro_shot().replace(n_phi=5, phi0=0.3, dphi=-0.07)
    assert np.array_equal(xrt.cell_mats(shot), o.cell_mats(shot))


def _call_simulate(st, fhkl=1, precision=0, image=1, dtype=0, acc=0):
    lib = xrt.load()
    return lib.xrt_simulate(C.byref(st.det), C.byref(st.beam), C.byref(st.xtal), C.c_void_p(fhkl),
                            precision, C.c_void_p(image), dtype, acc, None)


def err():
    return xrt.load().xrt_last_error().decode()


@pytest.mark.parametrize("field,value,code", [
    ("pixel", 0.0, xrt.XRT_EINVAL),
    ("distance", float("nan"), xrt.XRT_EINVAL),
    ("oversample", 0, xrt.XRT_ERANGE),
    ("n_layers", 3, xrt.XRT_EINVAL),        # layer_dt == 0 with 3 layers
    ("roi_f1", 129, xrt.XRT_EINVAL),
    ("roi_s0", 128, xrt.XRT_EINVAL),
    ("roi_f1", 0, xrt.XRT_EINVAL),          # empty region: f0 == f1
    ("roi_s1", 0, xrt.XRT_EINVAL),          # empty region: s0 == s1
])
def test_detector_validation(field, value, code):
    st = xrt.ShotStructs(synth.tiny_shot())
    setattr(st.det, field, value)
    assert _call_simulate(st) == code
    assert err()


def test_struct_size_mismatch():
    st = xrt.ShotStructs(synth.tiny_shot())
    st.xtal.struct_size -= 8
    assert _call_simulate(st) == xrt.XRT_EVERSION
    assert "struct_size" in err()


def test_crystal_validation():
    st = xrt.ShotStructs(synth.tiny_shot())
    st.xtal.N[1] = 5.5  # sincg needs whole cells
    assert _call_simulate(st) == xrt.XRT_EINVAL
    st = xrt.ShotStructs(synth.tiny_shot().replace(shape=synth.SHAPE_GAUSS))
    st.xtal.N[1] = 5.5
    # the Gaussian shape accepts real N: validation passes, the NULL table fails
    assert _call_simulate(st, fhkl=0) == xrt.XRT_EINVAL
    assert "fhkl" in err()
    st.xtal.N[0] = 0.0
    assert _call_simulate(st) == xrt.XRT_ERANGE
    st = xrt.ShotStructs(synth.tiny_shot())
    st.xtal.umats = None
    assert _call_simulate(st) == xrt.XRT_EINVAL


def test_beam_validation():
    shot = synth.tiny_shot()
    st = xrt.ShotStructs(shot.replace(src_lambda=np.array([-1.0])))
    assert _call_simulate(st) == xrt.XRT_EINVAL
    st = xrt.ShotStructs(shot.replace(evec=np.array([0.0, 0.0, 1.0])))  # along the beam
    assert _call_simulate(st) == xrt.XRT_EINVAL
    st = xrt.ShotStructs(shot.replace(src_dir=np.array([[0.0, 0.0, 2.0]])))
    assert _call_simulate(st) == xrt.XRT_EINVAL
    st = xrt.ShotStructs(shot)
    st.beam.n_src = 0  # no sources: an empty sum is refused, not silently zero
    assert _call_simulate(st) == xrt.XRT_ERANGE
    st = xrt.ShotStructs(shot)
    st.xtal.n_mos = 0
    assert _call_simulate(st) == xrt.XRT_EINVAL


def test_call_validation():
    st = xrt.ShotStructs(synth.tiny_shot())
    assert _call_simulate(st, precision=7) == xrt.XRT_EINVAL
    assert _call_simulate(st, dtype=5) == xrt.XRT_EINVAL
    assert _call_simulate(st, acc=2) == xrt.XRT_EINVAL
    assert _call_simulate(st, image=0) == xrt.XRT_EINVAL


def _call_background(shot, stol, F, molecules=1.0e10, n=None, size=None, image=1, precision=0, acc=0):
    st = xrt.ShotStructs(shot, crystal=False)
    x, f = np.ascontiguousarray(stol, np.float64), np.ascontiguousarray(F, np.float64)
    d = xrt.BackgroundDesc(C.sizeof(xrt.BackgroundDesc) if size is None else size,
                           len(x) if n is None else n, x.ctypes.data_as(xrt._pd), f.ctypes.data_as(xrt._pd),
                           molecules)
    return xrt.load().xrt_simulate_background(C.byref(st.det), C.byref(st.beam), C.byref(d), precision,
                                              C.c_void_p(image), 0, acc, None)


def test_background_validation():
    """Every malformed curve is rejected on the host, before anything is
    enqueued."""
    shot = synth.tiny_shot()
    bg = synth.water_background()
    x, F = bg.stol, bg.F
    cases = [
        (dict(stol=x[:1], F=F[:1]), xrt.XRT_ERANGE),                       # one knot
        (dict(stol=np.linspace(0, 1, 1025), F=np.ones(1025)), xrt.XRT_ERANGE),
        (dict(stol=x[::-1].copy(), F=F), xrt.XRT_EINVAL),                  # decreasing
        (dict(stol=np.r_[x[:3], x[2:]], F=np.r_[F[:3], F[2:]]), xrt.XRT_EINVAL),  # repeated knot
        (dict(stol=x, F=np.r_[F[:-1], np.nan]), xrt.XRT_EINVAL),
        (dict(stol=x, F=F, molecules=-1.0), xrt.XRT_EINVAL),
        (dict(stol=x, F=F, molecules=float("inf")), xrt.XRT_EINVAL),
        (dict(stol=np.array([0.0, 1e-300]), F=np.array([0.0, 1.0])), xrt.XRT_EINVAL),  # slope overflows
        (dict(stol=np.array([0.0, 1e39]), F=np.array([0.0, 1.0])), xrt.XRT_ERANGE),    # not binary32
        (dict(stol=x, F=F, size=8), xrt.XRT_EVERSION),
        (dict(stol=x, F=F, image=0), xrt.XRT_EINVAL),
        (dict(stol=x, F=F, precision=3), xrt.XRT_EINVAL),
        (dict(stol=x, F=F, acc=2), xrt.XRT_EINVAL),
    ]
    for kw, code in cases:
        assert _call_background(shot, **kw) == code, (kw, err())
        assert err()
    st = xrt.ShotStructs(shot, crystal=False)
    assert xrt.load().xrt_simulate_background(C.byref(st.det), C.byref(st.beam), None, 0, C.c_void_p(1), 0, 0,
                                              None) == xrt.XRT_EINVAL
    bad = shot.replace(roi=(0, 129, 0, 128))
    assert _call_background(bad, x, F) == xrt.XRT_EINVAL


def test_add_image_validation():
    lib = xrt.load()
    ok = dict(acc=8, anf=10, ans=10, img=8, dt=0, nf=4, ns=4, f0=0, s0=0)

    def call(**kw):
        a = dict(ok, **kw)
        return lib.xrt_add_image(C.c_void_p(a["acc"]), a["anf"], a["ans"], C.c_void_p(a["img"]), a["dt"], a["nf"],
                                 a["ns"], a["f0"], a["s0"], None)
    for kw, code in [(dict(acc=0), xrt.XRT_EINVAL), (dict(img=0), xrt.XRT_EINVAL), (dict(dt=2), xrt.XRT_EINVAL),
                     (dict(nf=0), xrt.XRT_EINVAL), (dict(anf=-1), xrt.XRT_EINVAL),
                     (dict(f0=7), xrt.XRT_EINVAL), (dict(s0=-1), xrt.XRT_EINVAL), (dict(ns=11), xrt.XRT_EINVAL),
                     (dict(anf=2 ** 30, ans=2 ** 10), xrt.XRT_ERANGE)]:
        assert call(**kw) == code, kw
        assert err()


def test_add_images_validation():
    lib = xrt.load()
    ptrs = (C.c_void_p * 2)(8, 16)
    bad = (C.c_void_p * 2)(8, None)
    assert lib.xrt_add_images(None, 4, 4, ptrs, 0, 2, None) == xrt.XRT_EINVAL
    assert lib.xrt_add_images(C.c_void_p(8), 4, 4, ptrs, 3, 2, None) == xrt.XRT_EINVAL
    assert lib.xrt_add_images(C.c_void_p(8), 0, 4, ptrs, 0, 2, None) == xrt.XRT_EINVAL
    assert lib.xrt_add_images(C.c_void_p(8), 4, 4, ptrs, 0, -1, None) == xrt.XRT_ERANGE
    assert lib.xrt_add_images(C.c_void_p(8), 4, 4, None, 0, 2, None) == xrt.XRT_EINVAL
    assert lib.xrt_add_images(C.c_void_p(8), 4, 4, bad, 0, 2, None) == xrt.XRT_EINVAL
    assert "image 1" in err()
    assert lib.xrt_add_images(C.c_void_p(8), 4, 4, None, 0, 0, None) == xrt.XRT_OK  # nothing to add


def test_fhkl_create_validation():
    lib = xrt.load()
    h = C.c_void_p()
    d = xrt.FhklDesc(C.sizeof(xrt.FhklDesc), xrt._i3(-2, -2, -2), xrt._i3(5, 0, 5), xrt.XRT_F64, 0.0)
    assert lib.xrt_fhkl_create(C.byref(d), C.c_void_p(1), None, C.byref(h)) == xrt.XRT_EINVAL
    d = xrt.FhklDesc(C.sizeof(xrt.FhklDesc), xrt._i3(-2, -2, -2), xrt._i3(5, 5, 5), 9, 0.0)
    assert lib.xrt_fhkl_create(C.byref(d), C.c_void_p(1), None, C.byref(h)) == xrt.XRT_EINVAL
    d = xrt.FhklDesc(C.sizeof(xrt.FhklDesc), xrt._i3(-2, -2, -2), xrt._i3(5000, 5000, 50), xrt.XRT_F64, 0.0)
    assert lib.xrt_fhkl_create(C.byref(d), C.c_void_p(1), None, C.byref(h)) == xrt.XRT_ERANGE
    assert lib.xrt_fhkl_destroy(None) == 0


def test_trace_index_validation():
    shot = synth.micro_shot()
    with pytest.raises(xrt.XrtError) as e:
        xrt.trace_terms(shot, np.array([[0, 0, 4, 0, 0, 0]], np.int32))  # sub >= O^2
    assert e.value.code == xrt.XRT_ERANGE


def test_sinpi_validation():
    lib = xrt.load()
    assert lib.xrt_sinpi(C.c_void_p(8), -1, C.c_void_p(8), None, None) == xrt.XRT_ERANGE
    assert lib.xrt_sinpi(None, 4, C.c_void_p(8), None, None) == xrt.XRT_EINVAL
    assert lib.xrt_sinpi(C.c_void_p(8), 4, None, None, None) == xrt.XRT_EINVAL
    assert lib.xrt_sinpi(None, 0, None, None, None) == xrt.XRT_OK  # nothing to do, nothing launched


def test_exp_validation():
    lib = xrt.load()
    assert lib.xrt_exp(C.c_void_p(8), -1, C.c_void_p(8), None) == xrt.XRT_ERANGE
    assert lib.xrt_exp(None, 4, C.c_void_p(8), None) == xrt.XRT_EINVAL
    assert lib.xrt_exp(C.c_void_p(8), 4, None, None) == xrt.XRT_EINVAL
    assert lib.xrt_exp(None, 0, None, None) == xrt.XRT_OK


def test_header_is_plain_c(tmp_path):
    """include/xrt.h compiles as strict C99 on its own: no HIP, C++ or torch
    types leak into the boundary."""
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no host C compiler")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    src = tmp_path / "use.c"
    src.write_text('#include "include/xrt.h"\nint main(void) { xrt_detector d; (void)d; return XRT_OK; }\n')
    subprocess.run([cc, "-std=c99", "-pedantic", "-Wall", "-Wextra", "-Werror", "-I", root, "-c", str(src),
                    "-o", str(tmp_path / "use.o")], check=True)


def test_server_calls_reject_null():
    lib = xrt.load()
    assert lib.xrt_server_cancel(None, 1) == xrt.XRT_EINVAL
    assert lib.xrt_server_release(None, 1) == xrt.XRT_EINVAL
    assert lib.xrt_server_progress(None, None) == xrt.XRT_EINVAL
    assert lib.xrt_server_destroy(None) == xrt.XRT_OK
    p = C.c_void_p()
    assert lib.xrt_server_host_image(None, 1, C.byref(p)) == xrt.XRT_EINVAL


def test_server_desc_host_budget_range():
    """The host budget of write-out servers is validated before any device
    work: 0 (off) or [1 MiB, 1 TiB]."""
    lib = xrt.load()
    h = C.c_void_p()
    for budget in (1, (1 << 20) - 1, (1 << 40) + 1):
        d = xrt.ServerDesc(C.sizeof(xrt.ServerDesc), 1 << 30, 8, xrt.XRT_MIXED, xrt.XRT_SHAPE_SINCG, xrt.XRT_F32,
                           0, 5000.0, budget)
        assert lib.xrt_server_create(C.byref(d), C.c_void_p(8), C.byref(h)) == xrt.XRT_ERANGE
        assert "host_budget" in err()


def test_server_desc_segment_terms_range():
    """The segment size of served sums is validated before any device work:
    0 (the default) or [2^10, 2^40]; the descriptor's size names the field."""
    lib = xrt.load()
    h = C.c_void_p()
    for terms in (-1, 1, (1 << 10) - 1, (1 << 40) + 1):
        d = xrt.ServerDesc(C.sizeof(xrt.ServerDesc), 1 << 30, 8, xrt.XRT_MIXED, xrt.XRT_SHAPE_SINCG, xrt.XRT_F32,
                           0, 5000.0, 0, None, xrt.XRT_SERVE_SHORTEST_REMAINING, terms)
        assert lib.xrt_server_create(C.byref(d), C.c_void_p(8), C.byref(h)) == xrt.XRT_ERANGE
        assert "segment_terms" in err()
    d = xrt.ServerDesc(C.sizeof(xrt.ServerDesc) - 8, 1 << 30, 8, xrt.XRT_MIXED, xrt.XRT_SHAPE_SINCG, xrt.XRT_F32,
                       0, 5000.0, 0, None, xrt.XRT_SERVE_SHORTEST_REMAINING, 0)
    assert lib.xrt_server_create(C.byref(d), C.c_void_p(8), C.byref(h)) == xrt.XRT_EVERSION


def test_binding_fails_loudly_without_the_library(tmp_path):
    """With libxrt.so absent the binding raises instead of falling back to
    anything else (there is no CPU path in the product)."""
    import subprocess
    import sys
    code = ("import sys; sys.path.insert(0, %r)\n"
            "from paper_2205_07976_amd import xrt\n"
            "xrt.LIB_PATH = %r\n"
            "try:\n"
            "    xrt.load()\n"
            "except ImportError as e:\n"
            "    print('raised', e)\n" % (ROOT, str(tmp_path / "libxrt.so")))
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0 and "raised" in r.stdout and "missing" in r.stdout, r.stdout + r.stderr
