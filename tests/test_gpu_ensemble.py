"""Ensemble sums on the device: xrt_add_image against the plain definition
(``oracle/ensemble.py``), the images of served shots summed in a fixed order
against the standalone images summed in the same order, and the gradient of
shared crystal parameters reduced over several shots against the oracle's
per-shot gradients."""
import sys

import numpy as np
import pytest

import synth
from oracle import ensemble as ens
from oracle import oracle as o

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2205_07976_amd import refine, serve, xrt  # noqa: E402
from tests.test_gpu_adjoint import roi_pixels, small_roi_case  # noqa: E402


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_add_image_matches_definition(dtype):
    """Random placements, ragged sizes, a single pixel, the whole
    accumulator, whole rows, the four edges: bit for bit."""
    rng = np.random.default_rng(3)
    acc0 = rng.standard_normal((300, 517))
    # whole rows at 16-byte aligned starts take the four-pixels-per-lane path
    # (1-pixel tails at 517 x 37 and 517 x 1); 517 x 3 at row 11 starts 8
    # bytes off and takes the row path like the rest
    cases = [((1, 1), (0, 0)), ((517, 300), (0, 0)), ((19, 7), (498, 293)), ((300, 1), (217, 0)),
             ((1, 300), (0, 0)), ((257, 129), (100, 50)), ((64, 64), (453, 236)), ((517, 37), (0, 16)),
             ((517, 1), (0, 8)), ((517, 3), (0, 11))]
    acc = torch.as_tensor(acc0, device="cuda")
    ref = acc0
    for (nf, ns), (f0, s0) in cases:
        img = (rng.standard_normal((ns, nf)) * 1e3).astype(dtype)
        xrt.add_image(acc, torch.as_tensor(img, device="cuda"), (f0, s0))
        ref = ens.add_image(ref, img, f0, s0)
    torch.cuda.synchronize()
    assert np.array_equal(acc.cpu().numpy(), ref)


def test_ensemble_sum_in_order():
    rng = np.random.default_rng(4)
    shape = (120, 90)
    imgs = [rng.exponential(5.0, (40, 33)).astype(np.float32) for _ in range(12)]
    origins = [(int(rng.integers(0, 58)), int(rng.integers(0, 81))) for _ in range(12)]
    acc = torch.zeros(shape, dtype=torch.float64, device="cuda")
    for img, org in zip(imgs, origins):
        xrt.add_image(acc, torch.as_tensor(img, device="cuda"), org)
    torch.cuda.synchronize()
    assert np.array_equal(acc.cpu().numpy(), ens.ensemble_sum(shape, imgs, origins))


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("n", [1, 7, 300])
def test_add_images_in_one_pass(dtype, n):
    """n whole images in one call (300: two launches of up to 256) give the
    bits of n single-image calls in the same order and of the definition."""
    rng = np.random.default_rng(n)
    shape = (37, 53)
    acc0 = rng.standard_normal(shape)
    imgs = [(rng.standard_normal(shape) * 10.0 ** rng.integers(-3, 4)).astype(dtype) for _ in range(n)]
    timgs = [torch.as_tensor(im, device="cuda") for im in imgs]
    batch = torch.as_tensor(acc0, device="cuda")
    xrt.add_images(batch, timgs)
    one = torch.as_tensor(acc0, device="cuda")
    for im in timgs:
        xrt.add_image(one, im)
    torch.cuda.synchronize()
    assert torch.equal(batch, one)
    ref = acc0
    for im in imgs[:40]:  # the definition on the first 40 (the oracle's loops are slow)
        ref = ens.add_image(ref, im, 0, 0)
    part = torch.as_tensor(acc0, device="cuda")
    xrt.add_images(part, timgs[:40])
    torch.cuda.synchronize()
    assert np.array_equal(part.cpu().numpy(), ref)


def _small_served_shots(n, seed):
    """Served-stream shots (random orientation, 1-100 sources, 1-200 domains,
    N in [5, 40]) with their regions cut to at most 96 x 96 pixels."""
    base = synth.full_shot()
    rng = np.random.default_rng(seed)
    shots = []
    for _ in range(n):
        s = synth.served_shot(rng, base.F, base.hkl_min)
        f0, f1, s0, s1 = s.roi
        shots.append(s.replace(roi=(f0, min(f1, f0 + 96), s0, min(s1, s0 + 96))))
    return base, shots


def test_served_ensemble_equals_standalone():
    """Shots served together, each finished image added into a detector-size
    accumulator in ticket order, give the bits of the standalone images
    added in the same order."""
    base, shots = _small_served_shots(6, 21)
    fh = xrt.Fhkl.from_shot(base)
    srv = xrt.Server(fh, hbm_budget=1 << 30, max_resident=8, precision="mixed")
    acc = torch.zeros((base.n_slow, base.n_fast), dtype=torch.float64, device="cuda")
    imgs = serve.run_stream(srv, shots, np.zeros(len(shots)), keep=range(len(shots)))["images"]
    srv.close()
    for i, s in enumerate(shots):
        xrt.add_image(acc, imgs[i], (s.roi[0], s.roi[2]))
    ref = torch.zeros_like(acc)
    for s in shots:
        xrt.add_image(ref, xrt.simulate(s, fh, precision="mixed"), (s.roi[0], s.roi[2]))
    torch.cuda.synchronize()
    say("served ensemble: nonzero pixels", int((acc != 0).sum()))
    assert torch.equal(acc, ref)


def test_gradient_reduced_over_shots():
    """Three crystals of one cell (its rows C in the crystal frame, shared N
    and scale) in different orientations U_s: the gradient of
    L = sum_s sum_p g_sp I_sp with respect to C, N and the scale, through
    autograd over the per-shot adjoints, equals the sum over shots of the
    oracle's gradients chained by hand (dL/dc_i = sum_s U_s^T dL/d(U_s c_i))."""
    shot, origins, size = small_roi_case(n_roi=3, n_src=3, n_mos=4)
    fh = xrt.Fhkl.from_shot(shot)
    rng = np.random.default_rng(11)
    Us = [shot.U] + [synth.axis_angle_matrix(rng.standard_normal(3), 0.002 * (k + 1)) @ shot.U for k in range(2)]
    pix = roi_pixels(origins, size)
    gs = [rng.normal(size=len(pix)) for _ in Us]
    C = torch.tensor(shot.cell, dtype=torch.float64, device="cuda", requires_grad=True)
    N = torch.tensor(shot.N, dtype=torch.float64, device="cuda", requires_grad=True)
    sc = torch.tensor(1.0, dtype=torch.float64, device="cuda", requires_grad=True)
    L = 0.0
    for U, g in zip(Us, gs):
        M0 = (torch.as_tensor(U, device="cuda") @ C.T).T
        img = refine.gauss_rois(M0, N, sc, shot, fh, origins, size)
        L = L + (img * torch.as_tensor(g.reshape(img.shape), device="cuda")).sum()
    L.backward()
    ref_C, ref_N, ref_s = np.zeros((3, 3)), np.zeros(3), 0.0
    for U, g in zip(Us, gs):
        g13 = o.gradient(shot.replace(U=U), pix, g)
        ref_C += g13[:9].reshape(3, 3) @ U  # row i: U^T (dL/d(U c_i))
        ref_N += g13[9:12]
        ref_s += g13[12]
    got_C, got_N, got_s = C.grad.cpu().numpy(), N.grad.cpu().numpy(), float(sc.grad.cpu())
    say("C", got_C.ravel(), ref_C.ravel())
    say("N", got_N, ref_N, "scale", got_s, ref_s)
    assert np.all(np.abs(got_C - ref_C) <= 1e-10 * np.abs(ref_C).max())
    assert np.all(np.abs(got_N - ref_N) <= 1e-10 * np.abs(ref_N).max())
    assert abs(got_s - ref_s) <= 1e-10 * abs(ref_s)
