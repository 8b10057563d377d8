"""The regions-of-interest forward and the adjoint (Gaussian shape) against the
FP64 oracle and against central finite differences, through the C ABI."""
import math
import sys

import numpy as np
import pytest

import synth
from oracle import oracle as o
from tests.metrics import DBL_MIN, compare

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2205_07976_amd import refine, xrt  # noqa: E402


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def small_roi_case(n_roi=6, size=16, n_src=4, n_mos=5):
    """The refinement crystal and geometry with fewer sources and domains, so
    the oracle covers every pixel of the regions."""
    shot, origins = synth.roi_shot()
    shot = shot.replace(src_dir=shot.src_dir[::25][:n_src].copy(),
                        src_lambda=shot.src_lambda[::25][:n_src].copy(),
                        src_weight=shot.src_weight[::25][:n_src] / shot.src_weight[::25][:n_src].sum(),
                        umats=shot.umats[:n_mos].copy())
    origins = origins[:n_roi] + (32 - size) // 2
    return shot, origins.astype(np.int32), (size, size)


def roi_pixels(origins, roi_size):
    nf, ns = roi_size
    out = []
    for f0, s0 in origins:
        ss, ff = np.meshgrid(np.arange(s0, s0 + ns), np.arange(f0, f0 + nf), indexing="ij")
        out.append(np.stack([ff.ravel(), ss.ravel()], 1))
    return np.concatenate(out).astype(np.int32)


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("mixed", 1e-5)])
def test_rois_forward(precision, tol):
    shot, origins, size = small_roi_case()
    fh = xrt.Fhkl.from_shot(shot)
    img = xrt.simulate_rois(shot, fh, origins, size, precision=precision, out_dtype=torch.float64)
    torch.cuda.synchronize()
    ref = o.simulate(shot, roi_pixels(origins, size)).reshape(len(origins), size[1], size[0])
    r = compare(img.cpu().numpy(), ref, tiny=DBL_MIN)
    say("rois", precision, r, "peak", ref.max(), "smallest", ref[ref > 0].min())
    assert r["zeros_ok"] and r["max_rel"] <= tol and r["sub_abs"] <= tol
    # the regions sit on Bragg spots: their peaks are far above their edges
    assert np.median(ref.reshape(len(origins), -1).max(1) / np.maximum(ref[:, 0, 0], 1e-300)) > 100


def test_rois_sincg_and_ragged():
    """Regions whose size is not a multiple of the 16 x 16 tile, sincg shape."""
    shot = synth.tiny_shot().replace(oversample=2)
    origins = np.array([[0, 0], [100, 3], [40, 110], [77, 77]], np.int32)
    fh = xrt.Fhkl.from_shot(shot)
    img = xrt.simulate_rois(shot, fh, origins, (19, 13))
    torch.cuda.synchronize()
    ref = o.simulate(shot, roi_pixels(origins, (19, 13))).reshape(4, 13, 19)
    r = compare(img.cpu().numpy(), ref)
    assert r["zeros_ok"] and r["max_rel"] <= 1e-12


def _weights(n, seed=7):
    return np.random.default_rng(seed).normal(size=n)


def test_backward_matches_oracle_gradient():
    shot, origins, size = small_roi_case()
    fh = xrt.Fhkl.from_shot(shot)
    pix = roi_pixels(origins, size)
    g = _weights(len(pix))
    dLdI = torch.as_tensor(g.reshape(len(origins), size[1], size[0]), device="cuda")
    ref = o.gradient(shot, pix, g)
    g64 = xrt.backward_rois(shot, fh, origins, size, dLdI, "fp64").cpu().numpy()
    g64b = xrt.backward_rois(shot, fh, origins, size, dLdI, "fp64").cpu().numpy()
    g32 = xrt.backward_rois(shot, fh, origins, size, dLdI, "mixed").cpu().numpy()
    say("oracle", ref)
    say("fp64  ", g64)
    say("mixed ", g32)
    assert np.array_equal(g64, g64b)  # fixed-order reduction
    # M0 block: 9 components sharing one scale
    for sl in (slice(0, 9), slice(9, 12), slice(12, 13)):
        scale = np.max(np.abs(ref[sl]))
        assert np.all(np.abs(g64[sl] - ref[sl]) <= 1e-10 * scale), (g64[sl], ref[sl])
        assert np.all(np.abs(g32[sl] - ref[sl]) <= 1e-4 * scale), (g32[sl], ref[sl])


@pytest.fixture(scope="module")
def full_refinement():
    """The refinement workload at its full size: 512 regions of 32 x 32 pixels
    around predicted spots, 100 sources, 50 domains (60 000 terms per pixel),
    as the benchmark launches it; dL/dI is a seeded normal weight on the
    pixels of 12 seeded regions and zero on the other 500, so the oracle
    gradient (those 12 288 pixels, 7.4e8 terms) is the gradient of the whole
    launch."""
    shot, origins = synth.roi_shot()
    size = (32, 32)
    rng = np.random.default_rng(512)
    sel = np.sort(rng.choice(len(origins), 12, replace=False))
    dLdI = np.zeros((len(origins), size[1], size[0]))
    dLdI[sel] = rng.normal(size=(len(sel), size[1], size[0]))
    pix = roi_pixels(origins[sel], size)
    say(f"full refinement gradient: oracle over regions {sel.tolist()} ({len(pix)} pixels)")
    ref = o.gradient(shot, pix, dLdI[sel].reshape(-1))
    return shot, origins.astype(np.int32), size, torch.as_tensor(dLdI, device="cuda"), ref


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("mixed", 1e-4)])
def test_backward_full_launch_matches_oracle(full_refinement, precision, tol):
    """The full-size adjoint launch (2048 workgroups of partial sums, the
    fixed-order reduction over all of them) against the oracle gradient:
    binary64 to 1e-10 and mixed to 1e-4 of each group's largest component
    (M0, N, scale); a second launch gives the same bits."""
    shot, origins, size, dLdI, ref = full_refinement
    fh = xrt.Fhkl.from_shot(shot)
    say(f"backward_rois {precision}: {len(origins)} regions of {size}")
    g = xrt.backward_rois(shot, fh, origins, size, dLdI, precision).cpu().numpy()
    g2 = xrt.backward_rois(shot, fh, origins, size, dLdI, precision).cpu().numpy()
    assert np.array_equal(g, g2)
    say("oracle", ref)
    say(precision.ljust(6), g)
    for sl in (slice(0, 9), slice(9, 12), slice(12, 13)):
        scale = np.max(np.abs(ref[sl]))
        err = np.max(np.abs(g[sl] - ref[sl])) / scale
        say(f"  components {sl.start}-{sl.stop - 1}: max diff / max |ref| = {err:.3e}")
        assert err <= tol, (g[sl], ref[sl])


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_backward_binary32_residuals(precision):
    """dL/dI given in binary32 is converted exactly: the gradient equals the
    one from the same values in binary64, bit for bit."""
    shot, origins, size = small_roi_case(n_roi=4)
    fh = xrt.Fhkl.from_shot(shot)
    g = _weights(4 * size[0] * size[1], seed=13).astype(np.float32).reshape(4, size[1], size[0])
    g32 = torch.as_tensor(g, device="cuda")
    a = xrt.backward_rois(shot, fh, origins, size, g32, precision).cpu().numpy()
    b = xrt.backward_rois(shot, fh, origins, size, g32.double(), precision).cpu().numpy()
    assert np.array_equal(a, b)


def test_backward_matches_finite_differences():
    """Central differences (step 1e-6 relative) of L = sum g I through the GPU
    forward against the GPU adjoint."""
    shot, origins, size = small_roi_case(n_roi=3)
    fh = xrt.Fhkl.from_shot(shot)
    M0 = shot.U @ shot.cell.T  # columns U a_i
    base = shot.replace(U=np.eye(3), cell=M0.T.copy())
    g = _weights(len(origins) * size[0] * size[1], seed=9)
    gt = torch.as_tensor(g.reshape(len(origins), size[1], size[0]), device="cuda")

    def L(s):
        img = xrt.simulate_rois(s, fh, origins, size)
        torch.cuda.synchronize()
        return float((img.cpu().numpy().ravel() * g).sum())

    grad = xrt.backward_rois(base, fh, origins, size, gt).cpu().numpy()
    fd = np.zeros(13)
    for i in range(3):
        for c in range(3):
            h = 1e-6 * max(abs(base.cell[i, c]), 1.0)
            cp, cm = base.cell.copy(), base.cell.copy()
            cp[i, c] += h
            cm[i, c] -= h
            fd[3 * i + c] = (L(base.replace(cell=cp)) - L(base.replace(cell=cm))) / (2 * h)
    for i in range(3):
        h = 1e-6 * base.N[i]
        Np, Nm = base.N.copy(), base.N.copy()
        Np[i] += h
        Nm[i] -= h
        fd[9 + i] = (L(base.replace(N=Np)) - L(base.replace(N=Nm))) / (2 * h)
    fd[12] = (L(base.replace(scale=1 + 1e-6)) - L(base.replace(scale=1 - 1e-6))) / 2e-6
    say("adjoint", grad)
    say("fd     ", fd)
    for sl in (slice(0, 9), slice(9, 12), slice(12, 13)):
        scale = np.max(np.abs(fd[sl]))
        assert np.all(np.abs(grad[sl] - fd[sl]) <= 1e-5 * scale), (grad[sl], fd[sl])


def test_autograd_chain_to_physical_parameters():
    """torch.autograd through the adjoint to (a, b, c, beta, misorientation,
    N, scale) for the squared-residual loss against a noisy target made by the
    oracle at perturbed parameters, checked by central differences."""
    shot, origins, size = small_roi_case(n_roi=3)
    fh = xrt.Fhkl.from_shot(shot)
    abc0 = np.array([79.0, 79.0, 38.0])
    beta0 = math.radians(95.0)
    abc_t, beta_t, N_t, th_t, s_t = refine.perturbed(abc0, beta0, shot.N, 1.0)
    Mt = refine.m0_from_params(torch.tensor(abc_t), torch.tensor(beta_t), torch.tensor(th_t),
                               shot.U).numpy()
    tshot = shot.replace(U=np.eye(3), cell=Mt, N=N_t, scale=s_t)
    pix = roi_pixels(origins, size)
    clean = o.simulate(tshot, pix)
    rng = np.random.default_rng(5)
    k = 1e4 / clean.max()
    target = torch.as_tensor((rng.poisson(clean * k) / k).reshape(len(origins), size[1], size[0]),
                             device="cuda")

    def loss(params):
        abc, beta, th, N, s = params
        M0 = refine.m0_from_params(abc, beta, th, shot.U)
        img = refine.gauss_rois(M0, N, s, shot, fh, origins, size)
        return ((img - target) ** 2).sum()

    params = [torch.tensor(abc0, dtype=torch.float64, requires_grad=True),
              torch.tensor(beta0, dtype=torch.float64, requires_grad=True),
              torch.zeros(3, dtype=torch.float64, requires_grad=True),
              torch.tensor(shot.N, dtype=torch.float64, requires_grad=True),
              torch.tensor(1.0, dtype=torch.float64, requires_grad=True)]
    L0 = loss(params)
    L0.backward()
    auto = np.concatenate([p.grad.detach().cpu().numpy().ravel() for p in params])
    flat = np.concatenate([p.detach().cpu().numpy().ravel() for p in params])

    def unflat(x):
        return [torch.tensor(x[0:3]), torch.tensor(x[3]), torch.tensor(x[4:7]), torch.tensor(x[7:10]),
                torch.tensor(x[10])]

    fd = np.zeros_like(flat)
    for i in range(len(flat)):
        h = 1e-7 if i in (4, 5, 6) else 1e-6 * max(abs(flat[i]), 1.0)
        xp, xm = flat.copy(), flat.copy()
        xp[i] += h
        xm[i] -= h
        fd[i] = (float(loss(unflat(xp))) - float(loss(unflat(xm)))) / (2 * h)
    say("autograd", auto)
    say("fd      ", fd)
    assert np.all(np.abs(auto - fd) <= 1e-5 * np.abs(fd) + 1e-6 * np.max(np.abs(fd)))


def test_rois_split_sums():
    """Three 24 x 24 regions of the refinement workload (60 000 terms per
    pixel, 12 tiles in all, so each sum is cut into 58 parts): parity with the
    oracle, and the same bits as three one-region calls (which split into 58
    parts too)."""
    shot, origins = synth.roi_shot()
    origins = (origins[:3] + 4).astype(np.int32)
    size = (24, 24)
    fh = xrt.Fhkl.from_shot(shot)
    img = xrt.simulate_rois(shot, fh, origins, size, precision="fp64")
    ref = o.simulate(shot, roi_pixels(origins, size)).reshape(3, 24, 24)
    r = compare(img.cpu().numpy(), ref)
    say("rois split fp64", r)
    assert r["zeros_ok"] and r["max_rel"] <= 1e-12
    for k, (f0, s0) in enumerate(origins):
        one = xrt.simulate(shot, fh, precision="fp64", roi=(int(f0), int(f0) + 24, int(s0), int(s0) + 24))
        assert torch.equal(one, img[k])
