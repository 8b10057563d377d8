"""Closed forms and constructions used to pin the oracle.

These are textbook results written in a different form from the oracle's
(pixel coordinates instead of unit vectors, explicit reciprocal lattice), so a
mistake in the oracle does not cancel against the same mistake here.
"""
import math

import numpy as np

R_E = 2.8179403262e-15


def pixel_xyz(shot, i_f, i_s, u=0, v=0, t=0):
    """Lab position of a sample point for the axis-aligned detector (+x fast,
    +y slow, +z normal)."""
    O = shot.oversample
    x = (i_f + (v + 0.5) / O) * shot.pixel - shot.beam_f
    y = (i_s + (u + 0.5) / O) * shot.pixel - shot.beam_s
    z = shot.distance + t * shot.layer_dt
    return x, y, z


def flat_solid_angle(p, x, y, z):
    """Solid angle of a small p x p patch of a flat detector at (x, y, z) seen
    from the origin: p^2 z / R^3."""
    R = math.sqrt(x * x + y * y + z * z)
    return p * p * z / R ** 3


def kahn_xy(K, x, y, z):
    """Kahn factor for an on-axis beam polarised along x, in Cartesian form:
    (1 + z^2/R^2 - K (x^2 - y^2)/R^2) / 2."""
    R2 = x * x + y * y + z * z
    return 0.5 * (1.0 + z * z / R2 - K * (x * x - y * y) / R2)


def rotation_onto(a, b, twist=0.0):
    """A rotation taking the direction of a onto the direction of b, followed
    by a turn of `twist` radians about b."""
    a = np.asarray(a, float) / np.linalg.norm(a)
    b = np.asarray(b, float) / np.linalg.norm(b)
    v = np.cross(a, b)
    s = np.linalg.norm(v)
    c = float(a @ b)
    if s < 1e-15:
        R = np.eye(3) if c > 0 else -np.eye(3)
    else:
        k = v / s
        K = np.array([[0, -k[2], k[1]], [k[2], 0, -k[0]], [-k[1], k[0], 0]])
        R = np.eye(3) + s * K + (1 - c) * K @ K
    bt = np.array([[0, -b[2], b[1]], [b[2], 0, -b[0]], [-b[1], b[0], 0]])
    T = np.eye(3) + math.sin(twist) * bt + (1 - math.cos(twist)) * bt @ bt
    return T @ R


def bragg_orientation(shot, i_f, i_s, hkl, twist=0.3):
    """Wavelength and orientation U that put reflection hkl exactly in the
    diffraction condition at the centre of pixel (i_f, i_s): the scattering
    vector (d - z)/lambda there equals the reciprocal lattice vector of hkl."""
    x, y, z = pixel_xyz(shot, i_f, i_s)
    d = np.array([x, y, z]) / math.sqrt(x * x + y * y + z * z)
    q = d - np.array([0.0, 0.0, 1.0])
    # reciprocal vector in the crystal frame: cell @ s = hkl
    s_c = np.linalg.solve(np.asarray(shot.cell, float), np.asarray(hkl, float))
    lam = np.linalg.norm(q) / np.linalg.norm(s_c)
    U = rotation_onto(s_c, q, twist)
    return lam, U
