"""The kernels' sin(pi x) on the device (xrt_sinpi: the same device code the
lattice factor uses for sin(pi f) and sin(pi g), paper section II's
crystal-size transform), against references that share nothing with it:

* binary64 form: 6 x 2^24 seeded points and edge points of [0, 1/2] (about
  10^8) against sin computed on the host in 80-bit extended precision;
  odd symmetry exact;
* binary32 form: every normal binary32 value in [2^-126, 1/2] against the
  GPU's binary64 sin.  Subnormal inputs are left out: whether the device
  flushes them is a compiler mode, and the lattice factor never depends on
  them.

Error bounds, in ulp of the result, derived from the evaluation x * P(x^2):
the fit's relative error (2.1e-16 binary64, 4.2e-8 binary32: up to 1.9 and
0.7 ulp depending on where the value falls in its binade), the Horner steps
with fused multiply-adds (about 1 ulp: the last steps add to pi with mild
cancellation near x = 1/2), the rounding of x^2 (at most 0.3 ulp through
P) and of the final product (0.5 ulp): 4 ulp for binary64, 3 for binary32.
In relative terms that is under 1e-15 for binary64, far inside the 1e-12
pixel tolerance.  The measured maxima are printed."""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2205_07976_amd import xrt  # noqa: E402

PI_LD = np.longdouble("3.14159265358979323846264338327950288")
SINPI64_ULP = 4.0   # bounds derived in the module docstring
SINPI32_ULP = 3.0


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def ulp64(r):
    return np.spacing(np.abs(r).astype(np.float64))


def test_sinpi_binary64_against_extended_precision():
    """10^8 points: 6 seeded batches of 2^24 uniform on [0, 1/2] plus edge
    points, against sin in 80-bit extended precision (64-bit significand: the
    reference's own error is below 2^-11 binary64 ulp)."""
    assert np.finfo(np.longdouble).nmant >= 63, "needs 80-bit long double on the host"
    rng = np.random.default_rng(11)
    edge = np.array([0.0, 5e-324, 1e-300, 2.0 ** -32, 1e-8, 0.125, 0.25, 0.375, 0.4999999999999999, 0.5])
    worst, where, n = 0.0, 0.0, 0
    for b in range(6):
        x = rng.uniform(0.0, 0.5, 1 << 24)
        if b == 0:
            x = np.concatenate([edge, x])
        xd = torch.from_numpy(x).cuda()
        s64, _ = xrt.sinpi(xd)
        s = s64.cpu().numpy()
        ref = np.sin(PI_LD * x.astype(np.longdouble))
        err = np.abs(s.astype(np.longdouble) - ref)
        nz = ref != 0
        ulps = np.zeros_like(x)
        ulps[nz] = (err[nz] / ulp64(ref[nz]).astype(np.longdouble)).astype(np.float64)
        if b == 0:
            assert s[0] == 0.0
            # odd symmetry is exact: x * P(x^2) with x^2 even
            sn, _ = xrt.sinpi(-xd)
            assert torch.equal(sn, -s64)
        if ulps.max() > worst:
            worst, where = float(ulps.max()), float(x[np.argmax(ulps)])
        n += len(x)
    say("binary64 sinpi: max", worst, "ulp at x =", where, f"({n} points)")
    assert worst <= SINPI64_ULP


def test_sinpi_binary32_exhaustive():
    first = int(np.float32(2.0 ** -126).view(np.int32))
    top = int(np.float32(0.5).view(np.int32))
    worst, where = 0.0, 0.0
    chunk = 1 << 26
    for lo in range(first, top + 1, chunk):
        bits = torch.arange(lo, min(lo + chunk, top + 1), dtype=torch.int32, device="cuda")
        x32 = bits.view(torch.float32)
        x = x32.double()
        _, s32 = xrt.sinpi(x)
        ref = torch.sin(torch.pi * x)
        # binary32 ulp of the reference (all references here are normal)
        e = torch.floor(torch.log2(ref.abs()))
        ulp = torch.exp2(e - 23)
        u = ((s32.double() - ref).abs() / ulp)
        m = float(u.max())
        if m > worst:
            worst, where = m, float(x[int(u.argmax())])
    say("binary32 sinpi: max", worst, "ulp at x =", where, f"({top + 1 - first} inputs)")
    assert worst <= SINPI32_ULP


def test_exp_binary64_against_extended_precision():
    """The binary64 kernels' exp (Gaussian lattice factor) against 80-bit host
    exp on 2^21 seeded points of [-760, 45] (the lattice exponents lie in
    (-inf, log(Na^2 Nb^2 Nc^2)]), including the subnormal range and exact 0
    below it.  Bound: 2 ulp (the table entry's rounding and the last one,
    half an ulp each, the fit 0.01 ulp, the reduction less); a subnormal
    result is that value rounded once more to the subnormal grid: 2 ulp of
    the unrounded value (at most 2 spacings) + half a spacing."""
    assert np.finfo(np.longdouble).nmant >= 63, "needs 80-bit long double on the host"
    rng = np.random.default_rng(12)
    x = np.concatenate([rng.uniform(-760.0, 45.0, 1 << 21), rng.uniform(-2.0, 2.0, 1 << 16),
                        np.array([0.0, -0.0, 1e-300, -745.2, -745.1, -708.4, -708.3, 41.4, -1e4, -1e6])])
    y = xrt.exp(torch.from_numpy(x).cuda()).cpu().numpy()
    ref = np.exp(x.astype(np.longdouble))
    ref64 = ref.astype(np.float64)
    assert np.all(y[ref64 == 0] == 0)  # below the binary64 range: exactly 0
    nz = ref64 != 0
    err = np.abs(y[nz].astype(np.longdouble) - ref[nz])
    spacing = np.spacing(ref64[nz]).astype(np.longdouble)
    ulps = (err / spacing).astype(np.float64)
    normal = ref64[nz] >= np.finfo(np.float64).tiny
    say("binary64 exp: max", ulps[normal].max(), "ulp (normal results), max", ulps[~normal].max() if (~normal).any()
        else 0.0, "spacing (subnormal results)")
    assert ulps[normal].max() <= 2.0
    assert (~normal).sum() > 0 and ulps[~normal].max() <= 2.5
    assert y[x == 0.0][0] == 1.0
