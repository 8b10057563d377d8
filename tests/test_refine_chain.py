"""The host side of refinement (paper_2205_07976_amd/refine.py, the chain from
physical parameters to M0 that torch differentiates), on the CPU: the
monoclinic cell rows, the misorientation rotation against scipy's (an
independent routine), the composition, and its derivatives against finite
differences (torch.autograd.gradcheck)."""
import math

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

torch = pytest.importorskip("torch")

from paper_2205_07976_amd import refine  # noqa: E402


def t(x):
    return torch.tensor(x, dtype=torch.float64)


def test_monoclinic_rows():
    a, b, c, beta = 79.0, 81.0, 38.0, math.radians(95.0)
    rows = refine.monoclinic_rows(t(a), t(b), t(c), t(beta)).numpy()
    assert np.allclose(np.linalg.norm(rows, axis=1), [a, b, c], rtol=1e-15)
    cos_ac = rows[0] @ rows[2] / (a * c)
    assert abs(cos_ac - math.cos(beta)) < 1e-15
    assert abs(rows[0] @ rows[1]) < 1e-12 and abs(rows[1] @ rows[2]) < 1e-12
    ortho = refine.monoclinic_rows(t(a), t(b), t(c), t(math.pi / 2)).numpy()
    assert np.allclose(ortho, np.diag([a, b, c]), atol=1e-12)


def test_rotation_matches_scipy():
    rng = np.random.default_rng(3)
    for _ in range(20):
        th = rng.uniform(-math.pi, math.pi, 3)
        R = refine.rot_xyz(t(th)).numpy()
        ref = Rotation.from_euler("XYZ", th).as_matrix()  # intrinsic x, y', z'': Rx Ry Rz
        assert np.allclose(R, ref, atol=1e-14)
        assert np.allclose(R @ R.T, np.eye(3), atol=1e-14) and abs(np.linalg.det(R) - 1) < 1e-14


def test_m0_composition():
    rng = np.random.default_rng(4)
    U = Rotation.random(random_state=5).as_matrix()
    abc, beta = t([79.0, 79.0, 38.0]), t(math.radians(95.0))
    M0 = refine.m0_from_params(abc, beta, t([0.0, 0.0, 0.0]), U).numpy()
    rows = refine.monoclinic_rows(abc[0], abc[1], abc[2], beta).numpy()
    assert np.allclose(M0, (U @ rows.T).T, atol=1e-13)
    th = rng.uniform(-0.01, 0.01, 3)
    M0t = refine.m0_from_params(abc, beta, t(th), U).numpy()
    assert np.allclose(M0t, (Rotation.from_euler("XYZ", th).as_matrix() @ U @ rows.T).T, atol=1e-12)


def test_chain_derivatives():
    U = Rotation.random(random_state=6).as_matrix()

    def f(abc, beta, th):
        return refine.m0_from_params(abc, beta, th, U)

    inputs = (t([79.0, 80.0, 38.0]).requires_grad_(), t(math.radians(95.0)).requires_grad_(),
              t([0.01, -0.02, 0.003]).requires_grad_())
    assert torch.autograd.gradcheck(f, inputs, eps=1e-6, atol=1e-7, rtol=1e-6)
