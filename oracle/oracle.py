"""ctypes front-end of the FP64 CPU oracle (``xro.c``).

TEST INFRASTRUCTURE ONLY.  The tests, the smoke check and the benchmark's
CPU-baseline leg are its only users; the product path never imports it.  It
shares no code with the HIP library: it takes a ``synth.Shot`` (plain numpy
arrays) and hands it to its own C implementation.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "xro.c")
_LIB = os.path.join(_HERE, "libxro.so")

#: compile line of the oracle: no contraction and no fast-math, so the
#: operation sequence written in xro.c is the one executed
BUILD_CMD = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
             "-ffp-contract=off", "-fno-fast-math", "-Wall", "-o", _LIB, _SRC, "-lm"]


def build() -> str:
    subprocess.run(BUILD_CMD, check=True)
    return _LIB


_d3 = C.c_double * 3
_d9 = C.c_double * 9
_i3 = C.c_int32 * 3
_pd = C.POINTER(C.c_double)


class _Shot(C.Structure):
    _fields_ = [
        ("n_fast", C.c_int32), ("n_slow", C.c_int32),
        ("pixel", C.c_double), ("distance", C.c_double),
        ("beam_f", C.c_double), ("beam_s", C.c_double),
        ("fdet", _d3), ("sdet", _d3), ("odet", _d3),
        ("oversample", C.c_int32), ("n_layers", C.c_int32),
        ("layer_dt", C.c_double), ("atten_len", C.c_double),
        ("n_src", C.c_int32),
        ("src_dir", _pd), ("src_lambda", _pd), ("src_weight", _pd),
        ("fluence", C.c_double), ("kahn", C.c_double), ("evec", _d3),
        ("cell", _d9), ("U", _d9),
        ("n_mos", C.c_int32), ("umats", _pd),
        ("n_phi", C.c_int32), ("phi0", C.c_double), ("dphi", C.c_double),
        ("spindle", _d3), ("N", _d3), ("shape", C.c_int32),
        ("gauss_c", C.c_double), ("scale", C.c_double),
        ("hkl_min", _i3), ("hkl_count", _i3),
        ("F", _pd), ("F_default", C.c_double),
    ]


class _Bg(C.Structure):
    _fields_ = [("n_knots", C.c_int32), ("stol", _pd), ("F", _pd), ("molecules", C.c_double)]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        lib = C.CDLL(_LIB)
        lib.xro_simulate.argtypes = [C.POINTER(_Shot), C.c_int64, C.c_void_p, C.c_void_p, C.c_int]
        lib.xro_trace.argtypes = [C.POINTER(_Shot), C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p]
        lib.xro_cell_mats.argtypes = [C.POINTER(_Shot), C.c_void_p]
        lib.xro_lattice_sq.argtypes = [C.c_double, C.c_double, C.c_int32, C.c_double]
        lib.xro_lattice_sq.restype = C.c_double
        lib.xro_polarization.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_double]
        lib.xro_polarization.restype = C.c_double
        lib.xro_capture.argtypes = [C.c_int32, C.c_double, C.c_double, C.c_double]
        lib.xro_capture.restype = C.c_double
        lib.xro_gradient.argtypes = [C.POINTER(_Shot), C.c_int64, C.c_void_p, C.c_void_p,
                                     C.c_void_p, C.c_int]
        lib.xro_bg_curve.argtypes = [C.POINTER(_Bg), C.c_double]
        lib.xro_bg_curve.restype = C.c_double
        lib.xro_background.argtypes = [C.POINTER(_Shot), C.POINTER(_Bg), C.c_int64, C.c_void_p,
                                       C.c_void_p, C.c_int]
        _lib = lib
    return _lib


def _arr(x, dtype=np.float64):
    return np.ascontiguousarray(np.asarray(x, dtype=dtype))


class _Packed:
    """A C struct for one shot plus the arrays it points into (kept alive)."""

    def __init__(self, shot):
        self.keep = [_arr(shot.src_dir), _arr(shot.src_lambda), _arr(shot.src_weight),
                     _arr(shot.umats), _arr(shot.F)]
        sd, sl, sw, um, F = self.keep
        s = _Shot()
        s.n_fast, s.n_slow = shot.n_fast, shot.n_slow
        s.pixel, s.distance = shot.pixel, shot.distance
        s.beam_f, s.beam_s = shot.beam_f, shot.beam_s
        s.fdet, s.sdet, s.odet = _d3(*shot.fdet), _d3(*shot.sdet), _d3(*shot.odet)
        s.oversample, s.n_layers = shot.oversample, shot.n_layers
        s.layer_dt, s.atten_len = shot.layer_dt, shot.atten_len
        s.n_src = shot.n_src
        s.src_dir = sd.ctypes.data_as(_pd)
        s.src_lambda = sl.ctypes.data_as(_pd)
        s.src_weight = sw.ctypes.data_as(_pd)
        s.fluence, s.kahn, s.evec = shot.fluence, shot.kahn, _d3(*shot.evec)
        s.cell = _d9(*np.asarray(shot.cell, np.float64).ravel())
        s.U = _d9(*np.asarray(shot.U, np.float64).ravel())
        s.n_mos = shot.n_mos
        s.umats = um.ctypes.data_as(_pd)
        s.n_phi, s.phi0, s.dphi = shot.n_phi, shot.phi0, shot.dphi
        s.spindle, s.N = _d3(*shot.spindle), _d3(*shot.N)
        s.shape, s.gauss_c, s.scale = shot.shape, shot.gauss_c, shot.scale
        s.hkl_min = _i3(*[int(x) for x in shot.hkl_min])
        s.hkl_count = _i3(*F.shape)
        s.F = F.ctypes.data_as(_pd)
        s.F_default = shot.F_default
        self.s = s


def simulate(shot, pixels=None, nthreads: int = 0) -> np.ndarray:
    """FP64 image values.  ``pixels``: (n, 2) int32 (i_f, i_s) pairs; default
    the whole ROI, returned as a (rows, cols) image.  nthreads 0 = all cores."""
    lib = _load()
    pk = _Packed(shot)
    full = pixels is None
    pix = _arr(shot.pixel_list() if full else pixels, np.int32)
    out = np.empty(len(pix), np.float64)
    rc = lib.xro_simulate(C.byref(pk.s), len(pix), pix.ctypes.data, out.ctypes.data, int(nthreads))
    if rc != 0:
        raise MemoryError("oracle: allocation failed")
    return out.reshape(shot.roi_shape) if full else out


def trace(shot, idx):
    """S and h of single terms; idx: (n, 6) int32 (i_f, i_s, sub, layer, src, rot)."""
    lib = _load()
    pk = _Packed(shot)
    idx = _arr(idx, np.int32)
    S = np.empty((len(idx), 3))
    h = np.empty((len(idx), 3))
    if lib.xro_trace(C.byref(pk.s), len(idx), idx.ctypes.data, S.ctypes.data, h.ctypes.data):
        raise MemoryError("oracle: allocation failed")
    return S, h


def cell_mats(shot) -> np.ndarray:
    lib = _load()
    pk = _Packed(shot)
    out = np.empty((shot.n_phi * shot.n_mos, 3, 3))
    if lib.xro_cell_mats(C.byref(pk.s), out.ctypes.data):
        raise MemoryError("oracle: allocation failed")
    return out


def lattice_sq(h: float, N: float, shape: int, c: float = 0.63) -> float:
    return _load().xro_lattice_sq(float(h), float(N), int(shape), float(c))


def polarization(d, inc, e, K: float) -> float:
    d, inc, e = _arr(d), _arr(inc), _arr(e)
    return _load().xro_polarization(d.ctypes.data, inc.ctypes.data, e.ctypes.data, float(K))


def capture(t: int, dt: float, mu: float, cosrho: float) -> float:
    return _load().xro_capture(int(t), float(dt), float(mu), float(cosrho))


def gradient(shot, pixels, dLdI, nthreads: int = 0) -> np.ndarray:
    """13 FP64 values: dL/dM0 (3x3 row-major; M0 rows = U x cell rows),
    dL/dN (3), dL/dscale, for L = sum_p dLdI_p * I_p.  Gaussian shape only."""
    if shot.shape != 1:
        raise ValueError("oracle gradient is defined for the Gaussian shape")
    lib = _load()
    pk = _Packed(shot)
    pix = _arr(pixels, np.int32)
    g = _arr(dLdI)
    out = np.empty(13)
    if lib.xro_gradient(C.byref(pk.s), len(pix), pix.ctypes.data, g.ctypes.data,
                        out.ctypes.data, int(nthreads)):
        raise MemoryError("oracle: allocation failed")
    return out


class _PackedBg:
    def __init__(self, bg):
        self.keep = [_arr(bg.stol), _arr(bg.F)]
        b = _Bg()
        b.n_knots = len(self.keep[0])
        b.stol = self.keep[0].ctypes.data_as(_pd)
        b.F = self.keep[1].ctypes.data_as(_pd)
        b.molecules = float(bg.molecules)
        self.s = b


def bg_curve(bg, x) -> np.ndarray:
    """The scattering curve of a ``synth.Background`` at each stol of x."""
    lib = _load()
    pb = _PackedBg(bg)
    return np.array([lib.xro_bg_curve(C.byref(pb.s), float(v)) for v in np.ravel(x)])


def background(shot, bg, pixels=None, nthreads: int = 0) -> np.ndarray:
    """FP64 background of an amorphous scatterer (``synth.Background``) over
    the shot's detector and beam; ``pixels`` as for ``simulate``."""
    lib = _load()
    pk = _Packed(shot)
    pb = _PackedBg(bg)
    full = pixels is None
    pix = _arr(shot.pixel_list() if full else pixels, np.int32)
    out = np.empty(len(pix), np.float64)
    lib.xro_background(C.byref(pk.s), C.byref(pb.s), len(pix), pix.ctypes.data, out.ctypes.data,
                       int(nthreads))
    return out.reshape(shot.roi_shape) if full else out
