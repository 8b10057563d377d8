"""Pins of the FP64 oracle against what the physics fixes independently of it:
closed forms, exact invariants, special cases, quadrature sum rules, an
arbitrary-precision brute force and finite differences.  CPU only."""
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


# ---------------------------------------------------------------- pin 1 ----
@pytest.mark.parametrize("kahn", [0.0, 0.8])
@pytest.mark.parametrize("pix,hkl", [((90, 40), (2, -1, 3)), ((10, 117), (-1, 3, 0))])
def test_exact_bragg_peak(pix, hkl, kahn):
    """At an exact Bragg position every sincg factor sits at its limit N, so
    the pixel equals r_e^2 Phi s F^2 (Na Nb Nc)^2 P dOmega."""
    base = synth.tiny_shot().replace(N=np.array([5.0, 6.0, 7.0]), kahn=kahn)
    lam, U = geo.bragg_orientation(base, pix[0], pix[1], hkl)
    shot = base.replace(U=U, src_lambda=np.array([lam]))
    val = o.simulate(shot, np.array([pix], np.int32))[0]
    F = shot.F[hkl[0] + 20, hkl[1] + 20, hkl[2] + 20]
    x, y, z = geo.pixel_xyz(shot, *pix)
    expect = (geo.R_E ** 2 * shot.fluence * shot.scale * F * F * (5 * 6 * 7) ** 2
              * geo.kahn_xy(kahn, x, y, z) * geo.flat_solid_angle(shot.pixel, x, y, z))
    assert rel(val, expect) <= 1e-12


def test_direct_beam_zero_index():
    """On the direct beam S = 0 exactly, so every fractional index is 0 and
    each sincg factor takes its f = 0 limit N: with one on-axis source and one
    sample point per pixel the beam pixel is r_e^2 Phi s F(000)^2 (Na Nb Nc)^2
    dOmega (P = 1 at zero scattering angle).  The input generator's shot
    really puts S = 0 on the middle sub-pixel of pixel (16, 16)."""
    shot = synth.direct_beam_shot()
    idx = np.array([[16, 16, 4, 0, 0, r] for r in range(shot.n_phi * shot.n_mos)], np.int32)
    S, h = o.trace(shot, idx)
    assert np.all(S == 0.0) and np.all(h == 0.0)
    one = shot.replace(oversample=1, src_dir=shot.src_dir[:1], src_lambda=shot.src_lambda[:1],
                       src_weight=np.array([1.0]))
    val = o.simulate(one, np.array([[16, 16]], np.int32))[0]
    F = one.F[4, 4, 4]
    expect = (geo.R_E ** 2 * one.fluence * one.scale * F * F * (5 * 6 * 7) ** 2
              * geo.flat_solid_angle(one.pixel, 0.0, 0.0, one.distance))
    assert rel(val, expect) <= 1e-12


# ---------------------------------------------------------------- pin 2 ----
def test_unit_crystal_closed_form():
    """Na = Nb = Nc = 1 makes the lattice factor 1; with a constant structure
    factor the image is pure geometry: r_e^2 Phi s F^2 times the average over
    sub-pixels of sum over layers of dOmega * capture * P, in closed form."""
    rng = np.random.default_rng(3)
    shot = synth.Shot(
        n_fast=5, n_slow=3, pixel=1.5e-4, distance=0.08, beam_f=0.9e-3, beam_s=-0.2e-3,
        oversample=2, n_layers=2, layer_dt=1.0e-4, atten_len=1.2e-4,
        src_dir=np.array([[0, 0, 1.0], [0, 0, 1.0]]), src_lambda=np.array([1.2, 1.4]),
        src_weight=np.array([0.3, 0.7]), kahn=0.7,
        cell=synth.orthorhombic_cell(50, 60, 70), U=synth.random_rotation(rng),
        umats=np.stack([np.eye(3), synth.axis_angle_matrix([1, 2, 3], 0.01)]),
        N=np.array([1.0, 1.0, 1.0]), hkl_min=np.array([-2, -2, -2]),
        F=np.full((5, 5, 5), 3.0), F_default=3.0, fluence=2.5e23, scale=1.7)
    img = o.simulate(shot)
    expect = np.zeros_like(img)
    for i_s in range(3):
        for i_f in range(5):
            tot = 0.0
            for u in range(2):
                for v in range(2):
                    for t in range(2):
                        x, y, z = geo.pixel_xyz(shot, i_f, i_s, u, v, t)
                        R = math.sqrt(x * x + y * y + z * z)
                        cap = (math.exp(-t * 1e-4 * R / (1.2e-4 * z))
                               - math.exp(-(t + 1) * 1e-4 * R / (1.2e-4 * z)))
                        tot += geo.flat_solid_angle(shot.pixel, x, y, z) * cap * geo.kahn_xy(0.7, x, y, z)
            expect[i_s, i_f] = geo.R_E ** 2 * 2.5e23 * 1.7 * 9.0 * tot / 4.0
    assert rel(img, expect) <= 1e-13


# ---------------------------------------------------------------- pin 3 ----
@pytest.mark.parametrize("shape", [synth.SHAPE_SINCG, synth.SHAPE_GAUSS])
def test_friedel_bitwise(shape):
    """With a Friedel-symmetric table F(-h) = F(h), inverting the cell maps
    every h to -h exactly; rint and the lattice factor are odd/even exactly, so
    the image does not change in any bit."""
    shot = synth.tiny_shot().replace(shape=shape)
    a = o.simulate(shot)
    b = o.simulate(shot.replace(cell=-shot.cell))
    assert np.array_equal(a, b)
    assert a.max() > 0


# ---------------------------------------------------------------- pin 4 ----
def _rot_shot():
    rng = np.random.default_rng(11)
    p = 2.0 ** -13
    return synth.Shot(
        n_fast=16, n_slow=16, pixel=p, distance=2.0 ** -3, beam_f=8 * p, beam_s=8 * p,
        oversample=1, n_layers=2, layer_dt=2.0 ** -12, atten_len=1.2e-4,
        src_dir=np.array([[0, 0, 1.0]]), src_lambda=np.array([1.1]),
        src_weight=np.array([1.0]), kahn=0.0,
        cell=synth.orthorhombic_cell(400.0, 500.0, 600.0), U=synth.random_rotation(rng),
        umats=np.eye(3)[None].copy(), N=np.array([4.0, 5.0, 6.0]),
        hkl_min=np.array([-8, -8, -8]),
        F=synth.friedel_table(rng.uniform(1, 100, (17, 17, 17))), F_default=0.5)


def test_rotation_about_beam_bitwise():
    """Turning the crystal by 90 deg about the beam turns the image by 90 deg
    on a square, centred detector with exactly representable geometry: pixel
    (i_f, i_s) moves to (n-1-i_s, i_f) with every bit kept."""
    shot = _rot_shot()
    Rz = np.array([[0.0, -1.0, 0.0], [1.0, 0.0, 0.0], [0.0, 0.0, 1.0]])
    U2 = np.stack([-shot.U[1], shot.U[0], shot.U[2]])  # exactly Rz @ U
    assert np.array_equal(U2, Rz @ shot.U)
    a = o.simulate(shot)
    b = o.simulate(shot.replace(U=U2))
    n = 16
    moved = np.empty_like(a)
    for i_s in range(n):
        for i_f in range(n):
            moved[i_f, n - 1 - i_s] = a[i_s, i_f]
    assert np.array_equal(moved, b)
    assert len(np.unique(a)) > 100


# ---------------------------------------------------------------- pin 5 ----
def test_fluence_linear_bitwise():
    shot = synth.micro_shot()
    a = o.simulate(shot)
    b = o.simulate(shot.replace(fluence=2 * shot.fluence))
    assert np.array_equal(2 * a, b)


# ---------------------------------------------------------------- pin 6 ----
def test_splitting_identities():
    """One source of weight 1 equals two identical sources of weight 1/2; n
    identical mosaic domains equal one domain (domains are averaged)."""
    shot = synth.tiny_shot().replace(oversample=2)
    pix = synth.pixel_sample(shot, 200, 5)
    a = o.simulate(shot, pix)
    two = shot.replace(src_dir=np.repeat(shot.src_dir, 2, 0),
                       src_lambda=np.repeat(shot.src_lambda, 2),
                       src_weight=np.array([0.5, 0.5]))
    assert rel(o.simulate(two, pix), a) <= 1e-15
    many = shot.replace(umats=np.repeat(shot.umats, 7, 0))
    assert rel(o.simulate(many, pix), a) <= 1e-15


# ---------------------------------------------------------------- pin 7 ----
@pytest.mark.parametrize("cosrho", [1.0, 0.83, 0.45])
def test_capture_telescoping(cosrho):
    """Layers partition the sensor: their capture fractions add up to
    1 - exp(-T dt / (mu cos rho)), and successive layers fall off by the
    factor exp(-dt / (mu cos rho))."""
    dt, mu, T = 1.5e-4, 1.2e-4, 5
    c = [o.capture(t, dt, mu, cosrho) for t in range(T)]
    assert abs(sum(c) - (1 - math.exp(-T * dt / (mu * cosrho)))) <= 1e-15
    for t in range(1, T):
        assert c[t] / c[t - 1] == pytest.approx(math.exp(-dt / (mu * cosrho)), rel=1e-14)
    assert o.capture(0, 0.0, mu, cosrho) == 1.0


# ---------------------------------------------------------------- pin 8 ----
def test_polarization_special_cases():
    rng = np.random.default_rng(8)
    inc = np.array([0.0, 0.0, 1.0])
    e = np.array([1.0, 0.0, 0.0])
    for _ in range(20):
        d = rng.normal(size=3)
        d[2] = abs(d[2]) + 0.2
        d /= np.linalg.norm(d)
        c2 = d[2]
        # unpolarised: (1 + cos^2 2theta) / 2
        assert o.polarization(d, inc, e, 0.0) == pytest.approx((1 + c2 * c2) / 2, rel=1e-15)
        # linear in K
        p0, p1 = o.polarization(d, inc, e, 0.0), o.polarization(d, inc, e, 1.0)
        assert o.polarization(d, inc, e, 0.25) == pytest.approx(0.75 * p0 + 0.25 * p1, rel=1e-14)
    # fully polarised, scattering perpendicular to e (psi = 90 deg): P = 1
    d = np.array([0.0, math.sin(0.7), math.cos(0.7)])
    assert o.polarization(d, inc, e, 1.0) == pytest.approx(1.0, rel=1e-15)
    # fully polarised, scattering in the plane of e (psi = 0): P = cos^2 2theta
    d = np.array([math.sin(0.7), 0.0, math.cos(0.7)])
    assert o.polarization(d, inc, e, 1.0) == pytest.approx(math.cos(0.7) ** 2, rel=1e-14)
    # a tilted source: only the part of e perpendicular to it counts.  For
    # inc = (sin tau, 0, cos tau) and e = x that part is (cos tau, 0, -sin tau)
    # and inc x e_perp = y, written out in closed form; d at angle a from inc
    # and azimuth psi from e_perp gives P = (1 + cos^2 a - K cos 2psi sin^2 a)/2
    tau = 0.3
    inc2 = np.array([math.sin(tau), 0.0, math.cos(tau)])
    ep = np.array([math.cos(tau), 0.0, -math.sin(tau)])
    by = np.array([0.0, 1.0, 0.0])
    for a, psi, K in [(0.5, 0.0, 1.0), (0.5, math.pi / 2, 1.0), (0.8, 0.6, 1.0), (0.35, 2.2, 0.6),
                      (1.1, -0.9, 1.0)]:
        d = math.cos(a) * inc2 + math.sin(a) * (math.cos(psi) * ep + math.sin(psi) * by)
        expect = 0.5 * (1 + math.cos(a) ** 2 - K * math.cos(2 * psi) * math.sin(a) ** 2)
        assert o.polarization(d, inc2, e, K) == pytest.approx(expect, rel=1e-14, abs=1e-15)
    # psi = 0 with K = 1 is cos^2 2theta, psi = 90 deg is 1, for the tilted
    # source too (measuring psi from e itself instead of its perpendicular
    # part fails the psi = 90 deg case and the general ones above)
    d0 = math.cos(0.5) * inc2 + math.sin(0.5) * ep
    assert o.polarization(d0, inc2, e, 1.0) == pytest.approx(math.cos(0.5) ** 2, rel=1e-14)
    d90 = math.cos(0.5) * inc2 + math.sin(0.5) * by
    assert o.polarization(d90, inc2, e, 1.0) == pytest.approx(1.0, rel=1e-15)


# ---------------------------------------------------------------- pin 9 ----
@pytest.mark.parametrize("N", [1, 2, 5, 20, 37])
def test_sincg_sum_rule(N):
    """sin^2(pi N h)/sin^2(pi h) is a trigonometric polynomial of degree N-1
    (the Fejer kernel) whose mean over a period is N; the trapezoid rule with
    more than N nodes integrates it exactly."""
    M = 4 * N + 3
    vals = [o.lattice_sq(k / M + 0.123, N, synth.SHAPE_SINCG) for k in range(M)]
    assert sum(vals) / M == pytest.approx(N, rel=1e-13)
    # periodic in h and maximal (N^2) at integers
    assert o.lattice_sq(7.0, N, 0) == N * N
    assert o.lattice_sq(3.3, N, 0) == pytest.approx(o.lattice_sq(0.3, N, 0), rel=1e-12)
    if N > 1:
        assert o.lattice_sq(1.0 / N, N, 0) < 1e-25


@pytest.mark.parametrize("N", [5.0, 12.5, 20.0])
def test_gauss_sum_rule(N):
    """N^2 exp(-2 N^2 f^2/c) integrates to N sqrt(pi c / 2) over a period (the
    tails beyond |f| = 1/2 are below e^-19 for N >= 5)."""
    c = 0.63
    M = 20000
    vals = [o.lattice_sq((k + 0.5) / M - 0.5, N, synth.SHAPE_GAUSS, c) for k in range(M)]
    assert sum(vals) / M == pytest.approx(N * math.sqrt(math.pi * c / 2), rel=1e-8)


# --------------------------------------------------------------- pin 10 ----
@pytest.mark.parametrize("shape", [synth.SHAPE_SINCG, synth.SHAPE_GAUSS])
def test_brute_force_micro(shape):
    """Every loop longer than one, off-axis sources, partial polarization,
    phi steps, mosaic domains, the default F outside the table: the oracle
    agrees with a 50-digit brute force of the unreduced definitions."""
    shot = synth.micro_shot(shape=shape)
    pix = shot.pixel_list()
    a = o.simulate(shot, pix)
    b = np.array([float(x) for x in brute.simulate(shot, pix)])
    cond = np.array(brute.term_condition(shot, pix))
    tol = 2e-15 + 4 * cond
    assert np.all(np.abs(a - b) / b <= tol), (np.abs(a - b) / b, tol)
    assert np.all(np.abs(a - b) / b <= 1e-12)


def test_brute_force_tiny_pixels():
    """Single-term pixels of the 128 x 128 workload against the brute force;
    the tolerance follows each pixel's conditioning in h."""
    shot = synth.tiny_shot()
    pix = synth.pixel_sample(shot, 12, 21)
    a = o.simulate(shot, pix)
    b = np.array([float(x) for x in brute.simulate(shot, pix)])
    cond = np.array(brute.term_condition(shot, pix))
    assert np.all(np.abs(a - b) / b <= 2e-15 + 4 * cond)


def test_phi_steps_match_rotated_orientations():
    """n_phi spindle steps average the images of U replaced by R(phi_k) U,
    with R built by scipy (an independent rotation routine)."""
    from scipy.spatial.transform import Rotation
    shot = synth.micro_shot(shape=synth.SHAPE_GAUSS)
    pix = shot.pixel_list()
    both = o.simulate(shot, pix)
    parts = []
    for k in range(shot.n_phi):
        R = Rotation.from_rotvec(shot.spindle * (shot.phi0 + k * shot.dphi)).as_matrix()
        parts.append(o.simulate(shot.replace(U=R @ shot.U, n_phi=1, phi0=0.0, dphi=0.0), pix))
    assert rel(both, np.mean(parts, axis=0)) <= 1e-11


def test_default_outside_table():
    """A table that no reflection reaches behaves like a constant table equal
    to the default value."""
    shot = synth.micro_shot()
    far = shot.replace(hkl_min=np.array([100, 100, 100]))
    const = shot.replace(F=np.full_like(shot.F, shot.F_default))
    assert rel(o.simulate(far), o.simulate(const)) <= 1e-15


# --------------------------------------------------------------- pin 12 ----
def test_gradient_matches_finite_differences():
    """Analytic Gaussian gradient of L = sum g_p I_p against central
    differences in the cell matrix (with U = I it is the cell itself), in N
    and in the scale."""
    base = synth.micro_shot(shape=synth.SHAPE_GAUSS)
    M0 = base.U @ base.cell.T  # columns U a_i
    shot = base.replace(U=np.eye(3), cell=M0.T.copy(), N=np.array([6.0, 7.5, 9.0]))
    pix = shot.pixel_list()
    g = np.array([0.3, -1.2, 0.7, 2.0])

    def L(s):
        return float(g @ o.simulate(s, pix))

    grad = o.gradient(shot, pix, g)
    fd = np.zeros(13)
    for i in range(3):
        for c in range(3):
            h = 1e-6 * abs(shot.cell[i, c]) + 1e-9
            cp, cm = shot.cell.copy(), shot.cell.copy()
            cp[i, c] += h
            cm[i, c] -= h
            fd[3 * i + c] = (L(shot.replace(cell=cp)) - L(shot.replace(cell=cm))) / (2 * h)
    for i in range(3):
        h = 1e-6 * shot.N[i]
        Np, Nm = shot.N.copy(), shot.N.copy()
        Np[i] += h
        Nm[i] -= h
        fd[9 + i] = (L(shot.replace(N=Np)) - L(shot.replace(N=Nm))) / (2 * h)
    h = 1e-6
    fd[12] = (L(shot.replace(scale=1 + h)) - L(shot.replace(scale=1 - h))) / (2 * h)
    scale = np.max(np.abs(fd))
    assert np.all(np.abs(grad - fd) <= 1e-6 * scale + 1e-6 * np.abs(fd)), (grad, fd)
