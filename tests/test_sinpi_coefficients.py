"""The sin(pi x) and exp polynomials the kernels carry (paper_2205_07976_amd/csrc/
xrt_math.h), checked on the CPU against 50-digit mpmath: the coefficients as
stored, evaluated exactly, stay within the relative error the header states
(binary64 2.2e-16, binary32 4.3e-8) over a dense grid of [0, 1/2].  The
polynomial carries the lattice factor's sin(pi f) and sin(pi g) (the
crystal-size transform of paper section II)."""
import os
import re

import mpmath as mp
import pytest

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                      "paper_2205_07976_amd", "csrc", "xrt_math.h")


def coefficients(kind):
    """Horner coefficients, highest degree first, of the double or float
    sinpi_over_x in the header."""
    src = open(HEADER).read()
    sig = "double sinpi_over_x(double y, double c6" if kind == "f64" else "float sinpi_over_x(float y)"
    body = src[src.index(sig):]
    body = body[:body.index("return p;")]
    nums = re.findall(r"[-+]?\d+\.\d+(?:e[-+]?\d+)?", body)
    if kind == "f64":  # the first step's constant term is the named SINPI_C6
        c6 = re.search(r"constexpr double SINPI_C6 = ([-+]?\d+\.\d+(?:e[-+]?\d+)?);", src).group(1)
        nums.insert(1, c6)
    return [mp.mpf(float(n.rstrip("f"))) if kind == "f64" else mp.mpf(float(n)) for n in nums]


@pytest.mark.parametrize("kind,bound,degree", [("f64", 2.2e-16, 7), ("f32", 4.3e-8, 4)])
def test_stored_polynomial_error(kind, bound, degree):
    mp.mp.dps = 50
    cs = coefficients(kind)
    assert len(cs) == degree + 1
    if kind == "f32":  # the float literals are rounded to binary32 when compiled
        import numpy as np
        cs = [mp.mpf(float(np.float32(float(c)))) for c in cs]
    worst = mp.mpf(0)
    n = 4000
    for i in range(1, n + 1):
        x = mp.mpf(i) / (2 * n)
        p = mp.mpf(0)
        for c in cs:
            p = p * x * x + c
        worst = max(worst, abs(x * p / mp.sin(mp.pi * x) - 1))
    assert worst <= bound, float(worst)
    # near 0 the polynomial's constant term is pi to the storage precision
    assert abs(cs[-1] / mp.pi - 1) <= bound


def exp_coefficients():
    """Horner coefficients of exp(r) = 1 + r q(r), highest degree first: those
    of exp_q, then the final 1 that exp_f64 adds."""
    src = open(HEADER).read()
    body = src[src.index("double exp_q(double r)"):]
    body = body[body.index("double p = "):body.index("}")]
    return [mp.mpf(float(n)) for n in re.findall(r"[-+]?\d+\.\d+(?:e[-+]?\d+)?", body)] + [mp.mpf(1)]


def test_stored_exp_polynomial_error():
    """exp(r) on |r| <= ln2/2 (the reduced argument of the binary64 Gaussian
    lattice factor): the stored degree-11 polynomial, evaluated exactly, stays
    within 2.3e-17 relative of 50-digit exp."""
    mp.mp.dps = 50
    cs = exp_coefficients()
    assert len(cs) == 12 and cs[-1] == 1 and cs[-2] == 1
    r1 = mp.log(2) / 2
    worst = mp.mpf(0)
    n = 4000
    for i in range(n + 1):
        x = -r1 + 2 * r1 * i / n
        p = mp.mpf(0)
        for c in cs:
            p = p * x + c
        worst = max(worst, abs(p / mp.exp(x) - 1))
    assert worst <= 2.3e-17, float(worst)
