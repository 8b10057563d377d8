"""Pins of the oracle's background of an amorphous scatterer (air, water
around the crystal) against what the physics and the mathematics fix:
numpy's linear interpolation, closed forms in the scattering angle, the layer
and sub-pixel partitions, source additivity, a mirror symmetry and an
arbitrary-precision brute force.  CPU only."""
import math

import numpy as np
import pytest

import synth
from oracle import brute
from oracle import oracle as o
from tests import geometry as geo


def rel(a, b):
    a, b = np.asarray(a, float), np.asarray(b, float)
    return np.max(np.abs(a - b) / np.abs(b))


def one_pixel_shot(X=0.0, Y=0.0, D=0.1, p=1.0e-4, **kw):
    """A 1 x 1 detector whose pixel centre sits at (X, Y) from the foot of
    the perpendicular, an on-axis source at 1.3 A, one layer, O = 1."""
    base = synth.tiny_shot()
    args = dict(n_fast=1, n_slow=1, pixel=p, distance=D, beam_f=p / 2 - X, beam_s=p / 2 - Y,
                oversample=1, n_layers=1, layer_dt=0.0, roi=None)
    args.update(kw)
    return base.replace(**args)


def linear_curve(a, b, top=2.0, n=9, molecules=3.0e10):
    s = np.linspace(0.0, top, n)
    return synth.Background(stol=s, F=a + b * s, molecules=molecules)


# ---------------------------------------------------------------- curve ----
def test_curve_is_numpy_interp():
    """numpy.interp is the same piecewise-linear interpolant with constant
    extension: equal to rounding everywhere, exact at the knots."""
    bg = synth.water_background()
    rng = np.random.default_rng(1)
    x = np.concatenate([rng.uniform(-0.2, 1.5, 2000), bg.stol,
                        0.5 * (bg.stol[1:] + bg.stol[:-1]), [-1.0, 5.0]])
    got = o.bg_curve(bg, x)
    assert rel(got, np.interp(x, bg.stol, bg.F)) <= 4e-16
    assert np.array_equal(o.bg_curve(bg, bg.stol), bg.F)
    assert o.bg_curve(bg, [-3.0])[0] == bg.F[0] and o.bg_curve(bg, [9.0])[0] == bg.F[-1]


def test_curve_reproduces_lines():
    """Knots on a line reproduce the line between them."""
    bg = synth.Background(stol=np.sort(np.random.default_rng(2).uniform(0, 1, 30)),
                          F=None, molecules=1.0)
    bg.F = 1.5 - 0.75 * bg.stol
    x = np.linspace(bg.stol[0], bg.stol[-1], 777)
    assert rel(o.bg_curve(bg, x), 1.5 - 0.75 * x) <= 2e-15


# ----------------------------------------------------------- closed forms ----
def test_forward_pixel_closed_form():
    """A pixel on the beam axis: S = 0, so F_bg(0) = F_0, P = 1 and
    dOmega = p^2 / D^2."""
    bg = synth.water_background()
    shot = one_pixel_shot(fluence=3.0e23)
    val = o.background(shot, bg)[0, 0]
    expect = geo.R_E ** 2 * 3.0e23 * bg.molecules * bg.F[0] ** 2 * shot.pixel ** 2 / shot.distance ** 2
    assert rel(val, expect) <= 1e-15


@pytest.mark.parametrize("kahn", [0.0, 0.7])
@pytest.mark.parametrize("X,Y", [(0.03, 0.0), (0.0, 0.045), (0.02, -0.031)])
def test_scattering_angle_closed_form(kahn, X, Y):
    """At scattering angle 2theta (tan 2theta = r / D) the curve is read at
    sin(theta)/lambda; with a linear curve a + b stol, an on-axis beam
    polarised along x and weight w:
    I = r_e^2 Phi n w (a + b sin(theta)/lambda)^2 P dOmega."""
    lam, w = 1.3, 0.8
    bg = linear_curve(1.5, 4.0)
    shot = one_pixel_shot(X, Y, src_lambda=np.array([lam]), src_weight=np.array([w]), kahn=kahn)
    val = o.background(shot, bg)[0, 0]
    D = shot.distance
    theta = 0.5 * math.atan2(math.hypot(X, Y), D)
    F = 1.5 + 4.0 * math.sin(theta) / lam
    expect = (geo.R_E ** 2 * shot.fluence * bg.molecules * w * F * F
              * geo.kahn_xy(kahn, X, Y, D) * geo.flat_solid_angle(shot.pixel, X, Y, D))
    assert rel(val, expect) <= 1e-14


def test_layers_on_axis():
    """On the axis every layer sees the forward direction (S = 0, P = 1);
    layer t lies at D + t dt, so it adds the thin-sensor value times
    (D / (D + t dt))^2 and its Beer-Lambert fraction
    exp(-t dt / mu) - exp(-(t + 1) dt / mu)."""
    bg = synth.water_background()
    thin = o.background(one_pixel_shot(), bg)[0, 0]
    T, dt, mu, D = 4, 5.0e-5, 1.2e-4, 0.1
    thick = o.background(one_pixel_shot(n_layers=T, layer_dt=dt, atten_len=mu), bg)[0, 0]
    factor = sum((D / (D + t * dt)) ** 2 * (math.exp(-t * dt / mu) - math.exp(-(t + 1) * dt / mu))
                 for t in range(T))
    assert rel(thick, thin * factor) <= 1e-14


def test_subpixels_are_small_pixels():
    """Oversample O over pixels of pitch p equals the sum of the O^2 pixels
    of pitch p/O that tile it (dOmega of the full pixel, averaged by 1/O^2)."""
    bg = synth.water_background()
    base = synth.tiny_shot().replace(n_fast=6, n_slow=5, pixel=2.0e-3, distance=0.05,
                                     beam_f=-4.0e-3, beam_s=3.0e-3, roi=None, kahn=0.5)
    O = 3
    coarse = o.background(base.replace(oversample=O), bg)
    fine = o.background(base.replace(n_fast=6 * O, n_slow=5 * O, pixel=base.pixel / O, roi=None), bg)
    summed = fine.reshape(5, O, 6, O).sum(axis=(1, 3))
    assert rel(coarse, summed) <= 1e-14


def test_sources_add():
    """The background of a beam is the weighted sum over its sources."""
    bg = synth.air_background()
    shot = synth.micro_shot()
    pix = shot.pixel_list()
    total = o.background(shot, bg, pix)
    parts = 0.0
    for j in range(shot.n_src):
        one = shot.replace(src_dir=shot.src_dir[j:j + 1], src_lambda=shot.src_lambda[j:j + 1],
                           src_weight=shot.src_weight[j:j + 1])
        parts = parts + o.background(one, bg, pix)
    assert rel(total, parts) <= 1e-15


def test_scales_bitwise():
    bg = synth.water_background()
    shot = synth.micro_shot()
    a = o.background(shot, bg)
    assert np.array_equal(o.background(shot.replace(fluence=4 * shot.fluence), bg), 4 * a)
    bg2 = synth.Background(stol=bg.stol, F=bg.F, molecules=0.5 * bg.molecules)
    assert np.array_equal(o.background(shot, bg2), 0.5 * a)


def test_mirror_symmetry_bitwise():
    """Unpolarised on-axis beam, beam centre on a pixel corner of a square
    detector, one sample point per pixel: swapping the fast and slow indices
    swaps x and y of every direction and changes nothing else."""
    bg = synth.water_background()
    shot = synth.tiny_shot().replace(n_fast=40, n_slow=40, pixel=2.5e-3, distance=0.08,
                                     beam_f=0.05, beam_s=0.05, roi=None, kahn=0.0,
                                     n_layers=2, layer_dt=1.0e-4)
    img = o.background(shot, bg)
    assert np.array_equal(img, img.T)


# ------------------------------------------------------------ brute force ----
@pytest.mark.parametrize("bgname", ["water", "air"])
def test_brute_force(bgname):
    """Against the 50-digit brute force on a detector that spans the water
    ring (2theta from about 16 to 40 degrees), every loop longer than one."""
    bg = synth.water_background() if bgname == "water" else synth.air_background()
    shot = synth.micro_shot().replace(n_fast=3, n_slow=2, pixel=6.0e-3, beam_f=-1.4e-2,
                                      beam_s=-6.0e-3, roi=None)
    pix = shot.pixel_list()
    got = o.background(shot, bg, pix)
    want = np.array([float(x) for x in brute.background(shot, bg, pix)])
    assert rel(got, want) <= 1e-13
