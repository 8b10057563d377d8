"""Differentiable simulation of regions of interest (Gaussian shape).

The refinement of per-crystal parameters against measured images (paper
section II, "Scientific background": the model is refined until the simulated
image matches the measured one) needs dL/dparameters.  ``GaussRois`` wraps
xrt_simulate_rois / xrt_backward_rois in a torch.autograd.Function whose
inputs are M0 (rows U a, U b, U c: the cell in the lab frame before spindle
and mosaic rotations), N = (Na, Nb, Nc) and the scale; torch then chains to
physical parameters on the host (``m0_from_params``): cell lengths a, b, c,
the monoclinic angle beta and three small misorientation angles.
"""
from __future__ import annotations

import math

import numpy as np

from . import xrt


def monoclinic_rows(a, b, c, beta):
    """Rows a, b, c of a b-unique monoclinic cell in the crystal frame."""
    import torch
    z = torch.zeros_like(a)
    return torch.stack([torch.stack([a, z, z]), torch.stack([z, b, z]),
                        torch.stack([c * torch.cos(beta), z, c * torch.sin(beta)])])


def rot_xyz(theta):
    """R = Rx(t0) Ry(t1) Rz(t2)."""
    import torch
    one, zero = torch.ones_like(theta[0]), torch.zeros_like(theta[0])
    c, s = torch.cos(theta), torch.sin(theta)
    Rx = torch.stack([torch.stack([one, zero, zero]), torch.stack([zero, c[0], -s[0]]),
                      torch.stack([zero, s[0], c[0]])])
    Ry = torch.stack([torch.stack([c[1], zero, s[1]]), torch.stack([zero, one, zero]),
                      torch.stack([-s[1], zero, c[1]])])
    Rz = torch.stack([torch.stack([c[2], -s[2], zero]), torch.stack([s[2], c[2], zero]),
                      torch.stack([zero, zero, one])])
    return Rx @ Ry @ Rz


def m0_from_params(cell_abc, beta, theta, U):
    """M0 rows = R(theta) U cell_i(a, b, c, beta) (all torch, differentiable)."""
    import torch
    rows = monoclinic_rows(cell_abc[0], cell_abc[1], cell_abc[2], beta)
    U = torch.as_tensor(U, dtype=rows.dtype, device=rows.device)
    return (rot_xyz(theta) @ U @ rows.T).T


class _Ctx:
    """What the autograd function needs besides its tensor inputs."""

    def __init__(self, shot, fhkl, origins, roi_size, precision):
        self.shot = shot
        self.fhkl = fhkl
        self.origins = np.ascontiguousarray(np.asarray(origins, np.int32))
        self.roi_size = tuple(int(v) for v in roi_size)
        self.precision = precision

    def shot_for(self, M0, N, scale):
        M0 = np.asarray(M0, np.float64)
        return self.shot.replace(cell=M0.copy(), U=np.eye(3), N=np.asarray(N, np.float64).copy(),
                                 scale=float(scale))


def _gauss_rois_fn():
    import torch

    class GaussRois(torch.autograd.Function):
        """images[n_roi, ns, nf] = simulate(M0, N, scale); backward by the
        adjoint kernel (13 values, binary64)."""

        @staticmethod
        def forward(ctx, M0, N, scale, info):
            shot = info.shot_for(M0.detach().cpu().numpy(), N.detach().cpu().numpy(),
                                 float(scale.detach().cpu()))
            if shot.shape != 1:
                raise ValueError("GaussRois needs the Gaussian shape")
            img = xrt.simulate_rois(shot, info.fhkl, info.origins, info.roi_size, precision=info.precision,
                                    out_dtype=torch.float64)
            ctx.info = info
            ctx.shot = shot
            ctx.save_for_backward(M0, N, scale)
            return img

        @staticmethod
        def backward(ctx, g):
            M0, N, scale = ctx.saved_tensors
            info = ctx.info
            g13 = xrt.backward_rois(ctx.shot, info.fhkl, info.origins, info.roi_size,
                                    g.contiguous().to(torch.float64), precision=info.precision)
            g13 = g13.to(M0.device)
            return (g13[:9].reshape(3, 3).to(M0.dtype), g13[9:12].to(N.dtype),
                    g13[12].reshape(scale.shape).to(scale.dtype), None)

    return GaussRois


_FN = None


def gauss_rois(M0, N, scale, shot, fhkl, origins, roi_size, precision="fp64"):
    """Differentiable images of the regions of interest (Gaussian shape)."""
    global _FN
    if _FN is None:
        _FN = _gauss_rois_fn()
    return _FN.apply(M0, N, scale, _Ctx(shot, fhkl, origins, roi_size, precision))


def perturbed(cell_abc, beta, N, scale):
    """The perturbation of the refinement workload: cell lengths x1.002,
    beta + 0.1 deg, N -> 0.9 N, misorientation 0.02 deg about each axis,
    scale x1.2."""
    return (np.asarray(cell_abc) * 1.002, beta + math.radians(0.1), np.asarray(N) * 0.9,
            np.full(3, math.radians(0.02)), scale * 1.2)
