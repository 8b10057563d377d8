"""Seeded synthetic shots with the shapes of the paper's workload.

The paper (section II, "Scientific background") names what a simulated image
depends on: the crystal orientation, its composition from smaller crystals
(mosaic domains), the photon energy spectrum of the shot and one structure
factor per Bragg spot.  It prints no workload sizes, so the shapes below are
the stated synthetic stand-ins:

* ``tiny_shot``   128 x 128 pixels, one source, one mosaic domain, N = 5.
* ``full_shot``   2463 x 2527 pixels (a Pilatus-6M-sized panel), 100 sources,
                  50 mosaic domains, oversample 2, 3 sensor layers, N = 20,
                  Fhkl over [-60, 60]^3 with Wilson-like intensities.
* ``served_shot`` one shot of a served stream: random orientation, log-uniform
                  region of interest, 1-100 sources, 1-200 domains, N in [5, 40].
* ``micro_shot``  a 2 x 2 detector small enough for arbitrary-precision checks.

Conventions (shared by every consumer of a Shot):

* Units: metres for detector quantities, angstrom for wavelengths and the cell,
  radians for angles.
* Lab frame: beam along +z; detector fast axis +x, slow axis +y, normal +z.
* ``cell`` rows are the real-space vectors a, b, c in the crystal frame
  (a along x, b in the xy plane); ``U`` rotates the crystal frame into the lab.
* ``umats[m]`` is the lab-frame rotation of mosaic domain m.
* ``F`` is dense over h in [hkl_min[0], hkl_min[0] + F.shape[0]), and so on,
  with l fastest.

Random draws the method itself would make (mosaic axes and angles, spectrum)
are made here and handed to both sides as plain arrays.
"""
from __future__ import annotations

import dataclasses
import math
from dataclasses import dataclass, field

import numpy as np

SHAPE_SINCG = 0
SHAPE_GAUSS = 1

#: classical electron radius in metres (CODATA 2018)
R_E = 2.8179403262e-15


@dataclass
class Shot:
    # detector
    n_fast: int
    n_slow: int
    pixel: float
    distance: float
    beam_f: float
    beam_s: float
    fdet: np.ndarray = field(default_factory=lambda: np.array([1.0, 0.0, 0.0]))
    sdet: np.ndarray = field(default_factory=lambda: np.array([0.0, 1.0, 0.0]))
    odet: np.ndarray = field(default_factory=lambda: np.array([0.0, 0.0, 1.0]))
    oversample: int = 1
    n_layers: int = 1
    layer_dt: float = 0.0
    atten_len: float = 1.2e-4
    roi: tuple = None  # (f0, f1, s0, s1), half-open; None = whole detector
    # beam
    src_dir: np.ndarray = None      # (n_src, 3) propagation directions
    src_lambda: np.ndarray = None   # (n_src,) angstrom
    src_weight: np.ndarray = None   # (n_src,)
    fluence: float = 1.0e24         # photons / m^2
    kahn: float = 0.0
    evec: np.ndarray = field(default_factory=lambda: np.array([1.0, 0.0, 0.0]))
    # crystal
    cell: np.ndarray = None         # (3, 3) rows a, b, c (angstrom)
    U: np.ndarray = None            # (3, 3)
    umats: np.ndarray = None        # (n_mos, 3, 3)
    n_phi: int = 1
    phi0: float = 0.0
    dphi: float = 0.0
    spindle: np.ndarray = field(default_factory=lambda: np.array([0.0, 1.0, 0.0]))
    N: np.ndarray = field(default_factory=lambda: np.array([5.0, 5.0, 5.0]))
    shape: int = SHAPE_SINCG
    gauss_c: float = 0.63
    scale: float = 1.0
    # structure factors
    hkl_min: np.ndarray = None      # (3,) int
    F: np.ndarray = None            # (nh, nk, nl) float64
    F_default: float = 0.0

    def __post_init__(self):
        if self.roi is None:
            self.roi = (0, self.n_fast, 0, self.n_slow)
        self.roi = tuple(int(x) for x in self.roi)

    # ---- derived sizes -------------------------------------------------
    @property
    def n_src(self) -> int:
        return int(len(self.src_lambda))

    @property
    def n_mos(self) -> int:
        return int(self.umats.shape[0])

    @property
    def roi_shape(self) -> tuple:
        f0, f1, s0, s1 = self.roi
        return (s1 - s0, f1 - f0)

    @property
    def n_pixels(self) -> int:
        a, b = self.roi_shape
        return a * b

    @property
    def terms_per_pixel(self) -> int:
        return (self.oversample ** 2) * self.n_layers * self.n_src * self.n_mos * self.n_phi

    @property
    def n_terms(self) -> int:
        return self.n_pixels * self.terms_per_pixel

    def replace(self, **kw) -> "Shot":
        """A copy with some fields replaced (arrays are copied, not shared)."""
        d = {}
        for f in dataclasses.fields(self):
            v = getattr(self, f.name)
            d[f.name] = v.copy() if isinstance(v, np.ndarray) else v
        d.update(kw)
        return Shot(**d)

    def pixel_list(self) -> np.ndarray:
        """All (i_f, i_s) pairs of the ROI in row-major (slow, fast) order."""
        f0, f1, s0, s1 = self.roi
        ss, ff = np.meshgrid(np.arange(s0, s1), np.arange(f0, f1), indexing="ij")
        return np.stack([ff.ravel(), ss.ravel()], axis=1).astype(np.int32)


# ---------------------------------------------------------------------------
# small building blocks
# ---------------------------------------------------------------------------

def random_rotation(rng: np.random.Generator) -> np.ndarray:
    """Uniform rotation on SO(3): a normalised 4-D Gaussian is a uniform unit
    quaternion (Muller 1959 / Marsaglia 1972), mapped to its rotation matrix."""
    q = rng.standard_normal(4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
        [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
        [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)],
    ])


def axis_angle_matrix(axis, angle: float) -> np.ndarray:
    """Rotation by ``angle`` about the unit ``axis`` (right hand)."""
    u = np.asarray(axis, dtype=np.float64)
    u = u / np.linalg.norm(u)
    c, s = math.cos(angle), math.sin(angle)
    K = np.array([[0.0, -u[2], u[1]], [u[2], 0.0, -u[0]], [-u[1], u[0], 0.0]])
    return c * np.eye(3) + s * K + (1.0 - c) * np.outer(u, u)


def orthorhombic_cell(a: float, b: float, c: float) -> np.ndarray:
    return np.array([[a, 0.0, 0.0], [0.0, b, 0.0], [0.0, 0.0, c]])


def monoclinic_cell(a: float, b: float, c: float, beta_deg: float) -> np.ndarray:
    """b-unique monoclinic cell: a along x, b along y, c in the xz plane."""
    beta = math.radians(beta_deg)
    return np.array([[a, 0.0, 0.0], [0.0, b, 0.0],
                     [c * math.cos(beta), 0.0, c * math.sin(beta)]])


def friedel_table(F: np.ndarray) -> np.ndarray:
    """Make a table over a symmetric range [-n, n]^3 obey F(-h) = F(h): every
    entry takes the value of the member of its Friedel pair that is
    lexicographically non-negative."""
    nh, nk, nl = F.shape
    assert nh % 2 == 1 and nk % 2 == 1 and nl % 2 == 1
    h = np.arange(nh) - nh // 2
    k = np.arange(nk) - nk // 2
    l = np.arange(nl) - nl // 2
    H, K, L = np.meshgrid(h, k, l, indexing="ij")
    keep = (H > 0) | ((H == 0) & (K > 0)) | ((H == 0) & (K == 0) & (L >= 0))
    return np.where(keep, F, F[::-1, ::-1, ::-1]).copy()


def mosaic_umats(rng: np.random.Generator, n_mos: int, spread_deg: float) -> np.ndarray:
    """n_mos domain rotations: axes uniform on the sphere, angles N(0, spread)."""
    if n_mos == 1:
        return np.eye(3)[None].copy()
    axes = rng.standard_normal((n_mos, 3))
    axes /= np.linalg.norm(axes, axis=1, keepdims=True)
    angles = rng.normal(0.0, math.radians(spread_deg), n_mos)
    return np.stack([axis_angle_matrix(a, t) for a, t in zip(axes, angles)])


def gaussian_spectrum(rng: np.random.Generator, n_src: int, lam0: float, sigma: float):
    """Wavelengths drawn i.i.d. N(lam0, sigma) and sorted; weights from the
    Gaussian spectrum at each wavelength, normalised to sum 1."""
    if n_src == 1:
        return np.array([lam0]), np.array([1.0])
    lam = np.sort(rng.normal(lam0, sigma, n_src))
    w = np.exp(-((lam - lam0) ** 2) / (2.0 * sigma * sigma))
    return lam, w / w.sum()


def on_axis_sources(n_src: int) -> np.ndarray:
    d = np.zeros((n_src, 3))
    d[:, 2] = 1.0
    return d


def pixel_sample(shot: Shot, n: int, seed: int) -> np.ndarray:
    """A seeded subset of n distinct ROI pixels as (i_f, i_s) int32 pairs."""
    rng = np.random.Generator(np.random.PCG64(seed))
    f0, f1, s0, s1 = shot.roi
    total = (f1 - f0) * (s1 - s0)
    n = min(n, total)
    idx = np.sort(rng.choice(total, size=n, replace=False))
    nf = f1 - f0
    return np.stack([f0 + idx % nf, s0 + idx // nf], axis=1).astype(np.int32)


# ---------------------------------------------------------------------------
# workloads
# ---------------------------------------------------------------------------

def tiny_shot(seed: int = 1) -> Shot:
    """128 x 128 detector, 0.1 mm pixels at 100 mm, beam on centre; one source
    at 1.30 A; one domain, one phi step, oversample 1, one layer; orthorhombic
    50 x 60 x 70 A cell in a random orientation; sincg with N = 5; F uniform on
    [0, 1000] over [-20, 20]^3 (Friedel-symmetric), 0 outside; unpolarised."""
    rng = np.random.Generator(np.random.PCG64(seed))
    U = random_rotation(rng)
    F = friedel_table(rng.uniform(0.0, 1000.0, (41, 41, 41)))
    return Shot(
        n_fast=128, n_slow=128, pixel=1.0e-4, distance=0.1,
        beam_f=6.4e-3, beam_s=6.4e-3,
        oversample=1, n_layers=1, layer_dt=0.0,
        src_dir=on_axis_sources(1), src_lambda=np.array([1.30]), src_weight=np.array([1.0]),
        kahn=0.0,
        cell=orthorhombic_cell(50.0, 60.0, 70.0), U=U, umats=np.eye(3)[None].copy(),
        N=np.array([5.0, 5.0, 5.0]), shape=SHAPE_SINCG,
        hkl_min=np.array([-20, -20, -20]), F=F, F_default=0.0,
    )


def wilson_table(rng: np.random.Generator, n: int, mean_I: float = 1.0e5) -> np.ndarray:
    """Intensities ~ Exp(mean_I) (Wilson's acentric distribution), F = sqrt(I)
    rounded to FP32 so the same table is exact in both precisions."""
    I = rng.exponential(mean_I, (2 * n + 1,) * 3)
    F = np.sqrt(I).astype(np.float32).astype(np.float64)
    return friedel_table(F)


def full_shot(seed: int = 2, shape: int = SHAPE_SINCG, N: float = 20.0) -> Shot:
    """2463 x 2527 detector, 0.172 mm pixels at 150 mm, beam centred; 100
    sources with lambda ~ N(1.30, 0.003) A and Gaussian-spectrum weights; 50
    mosaic domains about random axes by N(0, 0.05 deg); oversample 2; 3 layers
    of 0.15 mm (attenuation length 0.12 mm); monoclinic 79 x 79 x 38 A,
    beta = 95 deg; N = 20; Fhkl over [-60, 60]^3 with Wilson intensities."""
    rng = np.random.Generator(np.random.PCG64(seed))
    U = random_rotation(rng)
    lam, w = gaussian_spectrum(rng, 100, 1.30, 0.003)
    umats = mosaic_umats(rng, 50, 0.05)
    F = wilson_table(rng, 60)
    p = 1.72e-4
    return Shot(
        n_fast=2463, n_slow=2527, pixel=p, distance=0.150,
        beam_f=2463 * p / 2.0, beam_s=2527 * p / 2.0,
        oversample=2, n_layers=3, layer_dt=1.5e-4, atten_len=1.2e-4,
        src_dir=on_axis_sources(100), src_lambda=lam, src_weight=w,
        kahn=0.0,
        cell=monoclinic_cell(79.0, 79.0, 38.0, 95.0), U=U, umats=umats,
        N=np.array([N, N, N]), shape=shape,
        hkl_min=np.array([-60, -60, -60]), F=F, F_default=0.0,
    )


def served_shot(rng: np.random.Generator, F: np.ndarray, hkl_min: np.ndarray) -> Shot:
    """One shot of a served stream sharing the full-size detector and table:
    random orientation; ROI sides log-uniform in [64, 2463] x [64, 2527] at a
    random offset; 1-100 sources; 1-200 domains; Na, Nb, Nc in [5, 40]."""
    p = 1.72e-4
    nf_det, ns_det = 2463, 2527
    U = random_rotation(rng)
    wf = int(round(math.exp(rng.uniform(math.log(64), math.log(nf_det)))))
    ws = int(round(math.exp(rng.uniform(math.log(64), math.log(ns_det)))))
    f0 = int(rng.integers(0, nf_det - wf + 1))
    s0 = int(rng.integers(0, ns_det - ws + 1))
    n_src = int(rng.integers(1, 101))
    n_mos = int(rng.integers(1, 201))
    lam, w = gaussian_spectrum(rng, n_src, 1.30, 0.003)
    umats = mosaic_umats(rng, n_mos, 0.05)
    N = rng.integers(5, 41, 3).astype(np.float64)
    return Shot(
        n_fast=nf_det, n_slow=ns_det, pixel=p, distance=0.150,
        beam_f=nf_det * p / 2.0, beam_s=ns_det * p / 2.0,
        oversample=2, n_layers=3, layer_dt=1.5e-4, atten_len=1.2e-4,
        roi=(f0, f0 + wf, s0, s0 + ws),
        src_dir=on_axis_sources(n_src), src_lambda=lam, src_weight=w,
        cell=monoclinic_cell(79.0, 79.0, 38.0, 95.0), U=U, umats=umats,
        N=N, shape=SHAPE_SINCG, hkl_min=np.asarray(hkl_min), F=F, F_default=0.0,
    )


def micro_shot(seed: int = 10, shape: int = SHAPE_SINCG) -> Shot:
    """2 x 2 detector with every loop of the sum longer than one: oversample 2,
    2 layers, 3 sources (two off-axis), 3 mosaic domains, 2 phi steps; partly
    polarised beam and a nonzero default structure factor."""
    rng = np.random.Generator(np.random.PCG64(seed))
    dirs = np.array([[0.0, 0.0, 1.0], [1e-3, 0.0, 1.0], [0.0, -2e-3, 1.0]])
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    ev = np.array([1.0, 0.0, 0.0])
    F = friedel_table(rng.uniform(10.0, 1000.0, (9, 9, 9)))
    return Shot(
        n_fast=2, n_slow=2, pixel=2.0e-3, distance=0.05,
        beam_f=-1.0e-3, beam_s=-1.5e-3,
        oversample=2, n_layers=2, layer_dt=1.0e-4, atten_len=1.2e-4,
        src_dir=dirs, src_lambda=np.array([1.29, 1.30, 1.31]),
        src_weight=np.array([0.25, 0.5, 0.25]), kahn=0.6, evec=ev,
        cell=orthorhombic_cell(50.0, 60.0, 70.0), U=random_rotation(rng),
        umats=mosaic_umats(rng, 3, 0.5), n_phi=2, phi0=0.01, dphi=0.02,
        spindle=np.array([0.0, 1.0, 0.0]),
        N=np.array([3.0, 4.0, 5.0]), shape=shape,
        hkl_min=np.array([-4, -4, -4]), F=F, F_default=7.0,
    )


def direct_beam_shot(seed: int = 12) -> Shot:
    """32 x 32 detector of 2^-13 m pixels at 2^-3 m, the beam through the
    centre of pixel (16, 16), oversample 3: the middle sub-pixel of that pixel
    lies exactly on the beam, so for the on-axis source its scattering vector
    is exactly 0 and so is every fractional index (h = 0: the lattice factor
    at its f = 0 limit); a second source off axis, 3 mosaic domains, 2 phi
    steps, N = (5, 6, 7)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    p = 2.0 ** -13
    dirs = np.array([[0.0, 0.0, 1.0], [1e-3, 0.0, 1.0]])
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    F = friedel_table(rng.uniform(10.0, 1000.0, (9, 9, 9)))
    return Shot(
        n_fast=32, n_slow=32, pixel=p, distance=0.125,
        beam_f=16.5 * p, beam_s=16.5 * p,
        oversample=3, n_layers=1, layer_dt=0.0,
        src_dir=dirs, src_lambda=np.array([1.30, 1.31]), src_weight=np.array([0.6, 0.4]),
        kahn=0.0,
        cell=orthorhombic_cell(50.0, 60.0, 70.0), U=random_rotation(rng),
        umats=mosaic_umats(rng, 3, 0.5), n_phi=2, phi0=0.01, dphi=0.02,
        spindle=np.array([0.0, 1.0, 0.0]),
        N=np.array([5.0, 6.0, 7.0]), shape=SHAPE_SINCG,
        hkl_min=np.array([-4, -4, -4]), F=F, F_default=0.0,
    )


def roi_shot(seed: int = 5, n_roi: int = 512, size: int = 32, lam0: float = 1.30):
    """The full-size crystal with the Gaussian shape (N = 20) and n_roi
    non-overlapping size x size regions of interest around its predicted
    Bragg spots: for every tabulated reflection the scattering vector
    S = (M0^T)^-1 h (M0 rows = U a, U b, U c) is tested against the Ewald
    sphere of lam0; the diffracted ray d = unit(S + z/lam0) is cut with the
    detector plane; spots are ranked by F^2 exp(-eps^2 / (2 sigma^2)) with eps
    the distance to the sphere and sigma = sqrt(c/2) / (N |a|) (the Gaussian's
    width in reciprocal space).  Returns (shot, origins[n_roi, 2] int32)."""
    shot = full_shot(seed=2, shape=SHAPE_GAUSS, N=20.0)
    M0 = shot.U @ shot.cell.T                      # columns U a_i
    B = np.linalg.inv(M0.T)                        # S = B h
    n = shot.F.shape[0] // 2
    r = np.arange(-n, n + 1)
    H = np.stack(np.meshgrid(r, r, r, indexing="ij"), -1).reshape(-1, 3).astype(np.float64)
    F = shot.F.reshape(-1)
    S = H @ B.T
    kout = S + np.array([0.0, 0.0, 1.0 / lam0])
    knorm = np.linalg.norm(kout, axis=1)
    eps = knorm - 1.0 / lam0
    sigma = math.sqrt(shot.gauss_c / 2.0) / (shot.N[0] * np.linalg.norm(shot.cell[0]))
    keep = np.abs(eps) < 6 * sigma
    d = kout[keep] / knorm[keep, None]
    score = (F[keep] ** 2) * np.exp(-eps[keep] ** 2 / (2 * sigma * sigma))
    fwd = d[:, 2] > 1e-3
    d, score = d[fwd], score[fwd]
    x = d[:, 0] * shot.distance / d[:, 2]
    y = d[:, 1] * shot.distance / d[:, 2]
    i_f = (x + shot.beam_f) / shot.pixel
    i_s = (y + shot.beam_s) / shot.pixel
    half = size // 2
    on = (i_f >= half) & (i_f < shot.n_fast - half) & (i_s >= half) & (i_s < shot.n_slow - half)
    order = np.argsort(-score[on], kind="stable")
    cf, cs = i_f[on][order], i_s[on][order]
    chosen = []
    occupied = []
    for fx, sx in zip(cf, cs):
        f0 = int(math.floor(fx)) - half
        s0 = int(math.floor(sx)) - half
        if any(abs(f0 - a) < size and abs(s0 - b) < size for a, b in occupied):
            continue
        occupied.append((f0, s0))
        chosen.append((f0, s0))
        if len(chosen) == n_roi:
            break
    if len(chosen) < n_roi:
        raise ValueError(f"only {len(chosen)} non-overlapping spots found")
    return shot, np.array(chosen, dtype=np.int32)


# ---------------------------------------------------------------------------
# background scatterers
# ---------------------------------------------------------------------------

@dataclass
class Background:
    """An amorphous scatterer around the crystal (air, water): a scattering
    curve given as knots (stol_k, F_k), stol = sin(theta)/lambda in 1/angstrom
    strictly increasing, F per molecule; and the number of molecules in the
    beam."""
    stol: np.ndarray
    F: np.ndarray
    molecules: float

    @property
    def n_knots(self) -> int:
        return int(len(self.stol))


def _knots(rng: np.random.Generator, n: int, top: float, power: float) -> np.ndarray:
    """n increasing knots on [0, top], denser at small stol (exponent power),
    each interior knot moved by up to a fifth of its gap (seeded)."""
    x = top * (np.arange(n) / (n - 1)) ** power
    gap = np.diff(x)
    x[1:-1] += rng.uniform(-0.2, 0.2, n - 2) * np.minimum(gap[:-1], gap[1:])
    return x


def water_background(seed: int = 7, n_knots: int = 48, molecules: float = 1.0e11) -> Background:
    """A liquid-water-like curve: a ring near stol = 0.16 / A (the 3.1 A
    oxygen-oxygen distance) on a slowly decaying base, knots on [0, 1.2] / A
    with a 2 % seeded jitter of the values.  A synthetic stand-in: the paper
    gives no background curve."""
    rng = np.random.Generator(np.random.PCG64(seed))
    s = _knots(rng, n_knots, 1.2, 1.5)
    F = (1.0 + 1.6 * np.exp(-(((s - 0.16) / 0.06) ** 2)) + 1.2 * np.exp(-((s / 0.6) ** 2)))
    F *= 1.0 + 0.02 * rng.uniform(-1.0, 1.0, n_knots)
    return Background(stol=s, F=F, molecules=molecules)


def air_background(seed: int = 8, n_knots: int = 24, molecules: float = 4.0e10) -> Background:
    """A gas-like curve: forward scattering of a 14-electron molecule falling
    off monotonically, knots on [0, 1.0] / A.  Synthetic, like
    water_background."""
    rng = np.random.Generator(np.random.PCG64(seed))
    s = _knots(rng, n_knots, 1.0, 1.3)
    F = 14.0 * np.exp(-((s / 0.35) ** 2)) + 0.5
    F *= 1.0 + 0.01 * rng.uniform(-1.0, 1.0, n_knots)
    return Background(stol=s, F=F, molecules=molecules)
