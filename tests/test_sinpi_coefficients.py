"""The sin(pi x) and exp polynomials and the exp table the kernels carry
(paper_2205_07976_amd/csrc/xrt_math.h), checked on the CPU against 50-digit
mpmath: the coefficients as stored, evaluated exactly, stay within the
relative error the header states (sin: binary64 2.2e-16, binary32 4.3e-8 over
a dense grid of [0, 1/2]); the table entries and reduction constants are the
correctly rounded binary64 values.  The sine carries the lattice factor's
sin(pi f) and sin(pi g), the exp its Gaussian form (the crystal-size
transform of paper section II) and the layer capture."""
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
    of exp_q, then the final 1 that exp_cw_f64 adds."""
    src = open(HEADER).read()
    body = src[src.index("double exp_q(double r)"):]
    body = body[body.index("double p = "):body.index("}")]
    return [mp.mpf(float(n)) for n in re.findall(r"[-+]?\d+\.\d+(?:e[-+]?\d+)?", body)] + [mp.mpf(1)]


def test_stored_exp_polynomial_error():
    """exp(r) on |r| <= ln2/2 (the reduced argument of the capture's exp and
    expm1): the stored degree-11 polynomial, evaluated exactly, stays within
    2.3e-17 relative of 50-digit exp."""
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


def exp_f64_source():
    src = open(HEADER).read()
    body = src[src.index("double exp_f64(double e, double c5"):]
    return src, body[:body.index("\n}")]


def test_table_exp_polynomial_error():
    """exp(r) on |r| <= ln2/128 (the reduced argument of the Gaussian lattice
    factor's table-driven exp): 1 + r q(r) with q's coefficients as stored
    (the named EXP_C5, then the three of the Horner steps, then 1), evaluated
    exactly, stays within 2.3e-18 relative of 50-digit exp."""
    mp.mp.dps = 50
    src, body = exp_f64_source()
    c5 = re.search(r"constexpr double EXP_C5 = ([-+]?\d+\.\d+(?:e[-+]?\d+)?);", src).group(1)
    steps = re.findall(r"fma_sc\(c5, r, ([-+]?\d+\.\d+(?:e[-+]?\d+)?)\)|fma_sc\(q, r, ([-+]?\d+\.\d+(?:e[-+]?\d+)?)\)",
                       body)
    cs = [mp.mpf(float(c5))] + [mp.mpf(float(a or b)) for a, b in steps]
    assert len(cs) == 4 and "__builtin_fma(q, r, 1.0)" in body
    cs += [mp.mpf(1), mp.mpf(1)]  # q's constant term, then exp(r) = 1 + r q(r)
    r1 = mp.log(2) / 128
    worst = mp.mpf(0)
    n = 4000
    for i in range(n + 1):
        x = -r1 + 2 * r1 * i / n
        p = mp.mpf(0)
        for c in cs:
            p = p * x + c
        worst = max(worst, abs(p / mp.exp(x) - 1))
    assert worst <= 2.3e-18, float(worst)


def test_exp_table_and_reduction_constants():
    """The 64 entries of EXP2_J64 are 2^(j/64) rounded to nearest binary64, and
    exp_f64's reduction constants are 64/ln2 rounded, and ln2/64 as a rounded
    head plus its rounded remainder (Cody and Waite's split)."""
    mp.mp.dps = 50
    src, body = exp_f64_source()
    tab = src[src.index("EXP2_J64[64] = {"):]
    tab = tab[:tab.index("};")]
    vals = [float.fromhex(x) for x in re.findall(r"0x[0-9a-f]\.[0-9a-f]+p[-+]\d+", tab)]
    assert len(vals) == 64
    for j, v in enumerate(vals):
        assert v == float(mp.power(2, mp.mpf(j) / 64)), j
    ln2_64 = mp.log(2) / 64
    k = re.search(r"__builtin_fma\(e, ([\d.e+-]+), SHIFT\)", body).group(1)
    hi, lo = re.findall(r"__builtin_fma\(-n, ([\d.e+-]+), (?:e|r)\)", body)
    assert float(k) == float(1 / ln2_64)
    assert float(hi) == float(ln2_64)
    assert float(lo) == float(ln2_64 - mp.mpf(float(hi)))
