"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Tolerances: binary64 path <= 1e-12 relative per pixel (max over pixels with
a nonzero reference; zero pixels must be zero); mixed path <= 1e-5.  S and h
must agree bit for bit, which is what keeps ill-conditioned single-term
pixels inside 1e-12.
"""
import sys
import time

import numpy as np
import pytest

import synth
from oracle import oracle as o
from tests.metrics import DBL_MIN, compare

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2205_07976_amd import xrt  # noqa: E402

FP64_TOL = 1e-12
MIXED_TOL = 1e-5


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def gpu_image(shot, precision="fp64", roi=None, fhkl=None, **kw):
    fh = fhkl or xrt.Fhkl.from_shot(shot)
    out = xrt.simulate(shot, fh, precision=precision, roi=roi, **kw)
    torch.cuda.synchronize()
    return out.cpu().numpy().astype(np.float64)


def random_terms(shot, n, seed):
    rng = np.random.default_rng(seed)
    f0, f1, s0, s1 = shot.roi
    cols = [rng.integers(f0, f1, n), rng.integers(s0, s1, n), rng.integers(0, shot.oversample ** 2, n),
            rng.integers(0, shot.n_layers, n), rng.integers(0, shot.n_src, n),
            rng.integers(0, shot.n_phi * shot.n_mos, n)]
    return np.stack(cols, 1).astype(np.int32)


# ------------------------------------------------------------------ S and h -
@pytest.mark.parametrize("name", ["tiny", "micro", "full"])
def test_trace_bitwise(name):
    shot = {"tiny": synth.tiny_shot, "micro": synth.micro_shot, "full": synth.full_shot}[name]()
    idx = random_terms(shot, 4096, 1)
    say(f"trace {name}: {len(idx)} terms")
    S_g, h_g = xrt.trace_terms(shot, idx)
    S_o, h_o = o.trace(shot, idx)
    assert np.array_equal(S_g, S_o)
    assert np.array_equal(h_g, h_o)


# ------------------------------------------------------- small full images --
@pytest.mark.parametrize("precision,tol", [("fp64", FP64_TOL), ("mixed", MIXED_TOL)])
def test_tiny_full_image(precision, tol):
    shot = synth.tiny_shot()
    say(f"tiny 128x128 {precision}")
    g = gpu_image(shot, precision)
    r = compare(g, o.simulate(shot))
    say(r)
    assert r["zeros_ok"] and r["max_rel"] <= tol


@pytest.mark.parametrize("shape", [synth.SHAPE_SINCG, synth.SHAPE_GAUSS])
@pytest.mark.parametrize("precision,tol", [("fp64", FP64_TOL), ("mixed", MIXED_TOL)])
def test_micro(shape, precision, tol):
    shot = synth.micro_shot(shape=shape)
    g = gpu_image(shot, precision)
    r = compare(g, o.simulate(shot))
    say("micro", shape, precision, r)
    assert r["zeros_ok"] and r["max_rel"] <= tol


def test_ragged_rois_and_single_pixel():
    """ROIs that end inside a tile, a single pixel and a single row."""
    shot = synth.tiny_shot().replace(oversample=3)
    fh = xrt.Fhkl.from_shot(shot)
    for roi in [(3, 48, 5, 42), (127, 128, 0, 1), (0, 128, 77, 78), (60, 61, 10, 100)]:
        g = gpu_image(shot, roi=roi, fhkl=fh)
        ref = o.simulate(shot.replace(roi=roi))
        r = compare(g, ref)
        say(roi, r)
        assert g.shape == ref.shape and r["zeros_ok"] and r["max_rel"] <= FP64_TOL


# ------------------------------------------------- full-size workload -------
@pytest.fixture(scope="module")
def full():
    shot = synth.full_shot()
    fh = xrt.Fhkl.from_shot(shot)
    say("full 2463x2527 fp64 launch")
    img64 = gpu_image(shot, "fp64", fhkl=fh)
    say("full 2463x2527 mixed launch")
    img32 = gpu_image(shot, "mixed", fhkl=fh)
    return shot, fh, img64, img32


def test_full_sampled_pixels(full):
    """The launch the benchmark times, checked at 256 seeded pixels."""
    shot, _, img64, img32 = full
    pix = synth.pixel_sample(shot, 256, 2024)
    ref = o.simulate(shot, pix)
    g64 = img64[pix[:, 1], pix[:, 0]]
    g32 = img32[pix[:, 1], pix[:, 0]]
    r64, r32 = compare(g64, ref), compare(g32, ref)
    say("full fp64", r64, "mixed", r32)
    assert r64["zeros_ok"] and r64["max_rel"] <= FP64_TOL
    assert r32["zeros_ok"] and r32["max_rel"] <= MIXED_TOL


def split_of(shot, n_tiles):
    """The split factor the library applies (its documented rule)."""
    n_outer = shot.oversample ** 2 * shot.n_layers * shot.n_src
    if n_tiles >= 2048:
        return 1
    k = min(-(-2048 // n_tiles), n_outer, n_outer * shot.n_phi * shot.n_mos // 1024, 64)
    return max(k, 1)


# 256 x 256 crops of the full-size shot: centred on the beam (pixel
# (1231.5, 1263.5) of the 2463 x 2527 detector) and at the corner of the last
# columns and first rows, whose last column is in the ragged last tile column
# of the full-size launch (2463 = 153 * 16 + 15)
CROPS = [(1103, 1359, 1135, 1391), (2207, 2463, 0, 256)]


@pytest.mark.parametrize("roi", CROPS, ids=["beam_centre", "corner"])
def test_full_crops(full, roi):
    """256 x 256 crops at the beam centre and at a corner, as windows of the
    full-size images (the benchmark's launch, whole sums) and as separate ROI
    launches (16 x 16 tiles, so each pixel's sum is split into 8 parts), in
    both precisions: every pixel against the oracle, and the two launches
    against each other to the rounding of a different summation order."""
    shot, fh, img64, img32 = full
    f0, f1, s0, s1 = roi
    say(f"crop {roi}: oracle on {(f1 - f0) * (s1 - s0)} pixels")
    ref = o.simulate(shot.replace(roi=roi))
    win64 = img64[s0:s1, f0:f1]
    win32 = img32[s0:s1, f0:f1]
    roi64 = gpu_image(shot, "fp64", roi=roi, fhkl=fh)
    roi32 = gpu_image(shot, "mixed", roi=roi, fhkl=fh)
    assert split_of(shot, 256) == 8
    for name, x, tol in [("win64", win64, FP64_TOL), ("roi64", roi64, FP64_TOL), ("win32", win32, MIXED_TOL),
                         ("roi32", roi32, MIXED_TOL)]:
        r = compare(x, ref)
        say(roi, name, r)
        assert r["zeros_ok"] and r["max_rel"] <= tol
    nz = win64 > 0
    assert np.array_equal(nz, roi64 > 0)
    assert np.max(np.abs(roi64[nz] - win64[nz]) / win64[nz]) <= 1e-13


@pytest.mark.parametrize("precision,tol", [("fp64", FP64_TOL), ("mixed", MIXED_TOL)])
def test_split_sums(full, precision, tol):
    """A 40 x 40 ROI of the full shot (9 tiles, so each pixel's 1200 outer
    iterations are cut into 58 parts): parity with the oracle, identical bits
    on a second call, and the accumulate option through the reduction."""
    shot, fh, img64, img32 = full
    roi = (1200, 1240, 1250, 1290)
    assert split_of(shot, 9) == 58
    ref = o.simulate(shot.replace(roi=roi))
    a = xrt.simulate(shot, fh, precision=precision, roi=roi, out_dtype=torch.float64)
    b = xrt.simulate(shot, fh, precision=precision, roi=roi, out_dtype=torch.float64)
    r = compare(a.cpu().numpy(), ref)
    say("split", precision, r)
    assert r["zeros_ok"] and r["max_rel"] <= tol
    assert torch.equal(a, b)
    xrt.simulate(shot, fh, precision=precision, roi=roi, out=b, accumulate=True)
    assert torch.equal(b, 2 * a)


def test_full_gauss_sampled():
    """A 200 x 64 region of the full-size crystal with the Gaussian shape
    (N = 20): its pixels span 285 decades (the lattice exponent reaches about
    -650 there), so the mixed form is stored in binary64 (a binary32 image
    holds nothing below 1.2e-38, which is 83 % of this region) and is held to
    the headline relative error on every pixel."""
    shot = synth.full_shot(shape=synth.SHAPE_GAUSS)
    roi = (900, 1100, 1500, 1564)
    g = gpu_image(shot, "fp64", roi=roi)
    ref = o.simulate(shot.replace(roi=roi))
    r = compare(g, ref)
    say("gauss fp64", r)
    assert r["zeros_ok"] and r["max_rel"] <= FP64_TOL
    m = gpu_image(shot, "mixed", roi=roi, out_dtype=torch.float64)
    rm = compare(m, ref, tiny=DBL_MIN)
    say("gauss mixed", rm, "smallest reference", ref[ref > 0].min())
    assert rm["n_resolved"] == ref.size  # no subnormal reference here
    assert rm["zeros_ok"] and rm["max_rel"] <= MIXED_TOL


# ------------------------------------------------------------ invariants ----
def test_invariants_bitwise():
    """Friedel (cell -> -cell), fluence doubling and repeat launches leave the
    GPU image unchanged in every bit, as they do the oracle's."""
    shot = synth.tiny_shot().replace(oversample=2)
    fh = xrt.Fhkl.from_shot(shot)
    for prec in ("fp64", "mixed"):
        a = gpu_image(shot, prec, fhkl=fh)
        assert np.array_equal(a, gpu_image(shot, prec, fhkl=fh))
        assert np.array_equal(a, gpu_image(shot.replace(cell=-shot.cell), prec, fhkl=fh))
        assert np.array_equal(2 * a, gpu_image(shot.replace(fluence=2 * shot.fluence), prec, fhkl=fh))


def test_rotation_about_beam_bitwise():
    from tests.test_oracle_pins import _rot_shot
    shot = _rot_shot()
    U2 = np.stack([-shot.U[1], shot.U[0], shot.U[2]])
    a = gpu_image(shot)
    b = gpu_image(shot.replace(U=U2))
    n = 16
    moved = np.empty_like(a)
    for i_s in range(n):
        for i_f in range(n):
            moved[i_f, n - 1 - i_s] = a[i_s, i_f]
    assert np.array_equal(moved, b)


def test_accumulate_and_output_types():
    """accumulate adds into the image (the fused add-image step) and the
    binary32 output is the rounded binary64 value."""
    shot = synth.tiny_shot()
    fh = xrt.Fhkl.from_shot(shot)
    base = torch.full((128, 128), 0.25, dtype=torch.float64, device="cuda")
    xrt.simulate(shot, fh, out=base, accumulate=True)
    once = gpu_image(shot, fhkl=fh)
    torch.cuda.synchronize()
    assert np.array_equal(base.cpu().numpy(), once + 0.25)
    f32 = gpu_image(shot, out_dtype=torch.float32, fhkl=fh)
    assert np.array_equal(f32, once.astype(np.float32).astype(np.float64))


def test_fhkl_f32_source_and_default():
    """A binary32 table and a table no reflection reaches (default only)."""
    shot = synth.micro_shot()
    fh32 = xrt.Fhkl.from_shot(shot, dtype=torch.float32)
    g = gpu_image(shot, fhkl=fh32)
    ref = o.simulate(shot.replace(F=shot.F.astype(np.float32).astype(np.float64)))
    assert compare(g, ref)["max_rel"] <= FP64_TOL
    far = shot.replace(hkl_min=np.array([100, 100, 100]))
    assert compare(gpu_image(far), o.simulate(far))["max_rel"] <= FP64_TOL


def test_extreme_N_and_unit_crystal():
    for N in ([1.0, 1.0, 1.0], [1000.0, 1.0, 37.0]):
        shot = synth.micro_shot().replace(N=np.array(N))
        r = compare(gpu_image(shot), o.simulate(shot))
        say(N, r)
        assert r["max_rel"] <= FP64_TOL


def test_exact_bragg_on_gpu():
    from tests import geometry as geo
    base = synth.tiny_shot().replace(N=np.array([5.0, 6.0, 7.0]))
    lam, U = geo.bragg_orientation(base, 90, 40, (2, -1, 3))
    shot = base.replace(U=U, src_lambda=np.array([lam]))
    g = gpu_image(shot, roi=(90, 91, 40, 41))[0, 0]
    x, y, z = geo.pixel_xyz(shot, 90, 40)
    F = shot.F[22, 19, 23]
    expect = (geo.R_E ** 2 * shot.fluence * F * F * (5 * 6 * 7) ** 2 * geo.kahn_xy(0.0, x, y, z)
              * geo.flat_solid_angle(shot.pixel, x, y, z))
    assert abs(g - expect) / expect <= FP64_TOL
    m = gpu_image(shot, "mixed", roi=(90, 91, 40, 41))[0, 0]
    assert abs(m - expect) / expect <= MIXED_TOL


@pytest.mark.parametrize("precision,tol", [("fp64", FP64_TOL), ("mixed", MIXED_TOL)])
def test_direct_beam_zero_index(precision, tol):
    """Terms whose fractional indices are exactly 0 (S = 0 on the direct
    beam): the ratio of sines is 0/0 there, and the kernels sum such a
    rotation loop again with the floored ratio.  The whole image (the beam
    pixel's on-axis sub-pixel takes that path, the rest do not) against the
    oracle, standalone and served; and with a single on-axis sample point the
    beam pixel against its closed form r_e^2 Phi F(000)^2 (Na Nb Nc)^2 dOmega."""
    shot = synth.direct_beam_shot()
    img = gpu_image(shot, precision)
    r = compare(img, o.simulate(shot))
    say("direct beam", precision, r)
    assert r["zeros_ok"] and r["max_rel"] <= tol
    srv = xrt.Server(xrt.Fhkl.from_shot(shot), hbm_budget=64 << 20, precision=precision)
    try:
        t = srv.submit(shot)
        deadline = time.monotonic() + 60.0
        while srv.progress() == 0:
            assert time.monotonic() < deadline, "served shot did not finish"
        served = srv.image(t).cpu().numpy().astype(np.float64)
        srv.release(t)
    finally:
        srv.close()
    assert np.array_equal(served, img)
    from tests import geometry as geo
    one = shot.replace(oversample=1, src_dir=shot.src_dir[:1], src_lambda=shot.src_lambda[:1],
                       src_weight=np.array([1.0]))
    g = gpu_image(one, precision, roi=(16, 17, 16, 17))[0, 0]
    F = one.F[4, 4, 4]
    expect = (geo.R_E ** 2 * one.fluence * F * F * (5 * 6 * 7) ** 2
              * geo.flat_solid_angle(one.pixel, 0.0, 0.0, one.distance))
    assert abs(g - expect) / expect <= tol


def test_clamped_index_path():
    """A cell so large that h leaves the padded table box: the kernels take
    the clamping index path (out-of-box reflections read F_default)."""
    base = synth.micro_shot()
    shot = base.replace(cell=8.0 * base.cell)
    S, h = o.trace(shot, random_terms(shot, 256, 3))
    assert np.abs(np.rint(h)).max() > 12  # beyond hkl range 4 + padding 8
    for prec, tol in (("fp64", FP64_TOL), ("mixed", MIXED_TOL)):
        r = compare(gpu_image(shot, prec), o.simulate(shot))
        say("clamp", prec, r)
        assert r["zeros_ok"] and r["max_rel"] <= tol
