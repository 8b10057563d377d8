"""Minimax fits of exp(r) for the binary64 exponentials of xrt_math.h.

exp_f64 (the Gaussian lattice factor) uses Tang's table-driven reduction:
e = (64 k + j) ln2/64 + r with j in [0, 64), exp(e) = 2^k 2^(j/64) exp(r) and
|r| <= ln2/128; exp(r) is a degree-5 polynomial there.  expm1_f64 uses
e = n ln2 + r, |r| <= ln2/2, and a degree-11 polynomial.  Both reductions
split the constant (ln2/64, ln2) into a binary64 head and tail (Cody and
Waite).  Each polynomial P(r) minimises the maximum relative error on its
interval, found by the Remez exchange algorithm in 50-digit mpmath, rounded
to binary64 and re-checked on a dense grid.  Run as a script to print the
coefficients, the reduction constants and the table of 2^(j/64), each
rounded to nearest binary64, that xrt_math.h carries:

    python fit_exp.py 11 1    # expm1_f64: degree 11 on |r| <= ln2/2
    python fit_exp.py 5 64    # exp_f64: degree 5 on |r| <= ln2/128, table
"""
from __future__ import annotations

import sys

import mpmath as mp

mp.mp.dps = 50
R1 = mp.log(2) / 2


def remez(deg: int, iters: int = 40):
    """Coefficients c_0..c_deg of the relative-minimax P on [-R1, R1]."""
    n = deg + 2
    xs = [-R1 * mp.cos(mp.pi * i / (n - 1)) for i in range(n)]
    E = mp.mpf(0)
    for _ in range(iters):
        A = mp.matrix(n, n)
        b = mp.matrix(n, 1)
        for i, x in enumerate(xs):
            t = mp.exp(x)
            for j in range(deg + 1):
                A[i, j] = x ** j
            A[i, deg + 1] = (-1) ** i * t
            b[i] = t
        sol = mp.lu_solve(A, b)
        c = [sol[j] for j in range(deg + 1)]
        E = sol[deg + 1]

        def err(y):
            return (mp.polyval(c[::-1], y) - mp.exp(y)) / mp.exp(y)
        grid = [-R1 + 2 * R1 * i / 4000 for i in range(4001)]
        vals = [err(y) for y in grid]
        ext = []
        i = 0
        while i < len(grid):
            j = i
            while j + 1 < len(grid) and mp.sign(vals[j + 1]) == mp.sign(vals[i]):
                j += 1
            k = max(range(i, j + 1), key=lambda q: abs(vals[q]))
            ext.append(grid[k])
            i = j + 1
        if len(ext) >= n:
            while len(ext) > n:
                a0, a1 = abs(err(ext[0])), abs(err(ext[-1]))
                ext.pop(0 if a0 < a1 else -1)
            xs = ext
    return c, abs(E)


def max_rel_err(coeffs, n=20001):
    """Max relative error of P with the coefficients rounded to binary64,
    evaluated exactly (isolates the fit and the coefficient rounding)."""
    cs = [mp.mpf(float(c)) for c in coeffs]
    worst = mp.mpf(0)
    for i in range(n):
        x = -R1 + 2 * R1 * i / (n - 1)
        worst = max(worst, abs(mp.polyval(cs[::-1], x) / mp.exp(x) - 1))
    return worst


if __name__ == "__main__":
    deg = int(sys.argv[1]) if len(sys.argv) > 1 else 11
    steps = int(sys.argv[2]) if len(sys.argv) > 2 else 1  # table entries per octave
    R1 = mp.log(2) / (2 * steps)
    c, E = remez(deg)
    print(f"degree {deg}: minimax relative error {mp.nstr(E, 4)}, "
          f"after rounding {mp.nstr(max_rel_err(c), 4)}")
    for k in range(deg, -1, -1):
        print(f"  c{k} = {float(c[k])!r}")
    ln2 = mp.log(2) / steps
    hi = float(ln2)
    print(f"ln2/{steps} head {hi!r}, tail {float(ln2 - mp.mpf(hi))!r}, {steps}/ln2 {float(1 / ln2)!r}")
    if steps > 1:
        tab = [float(mp.power(2, mp.mpf(j) / steps)) for j in range(steps)]
        for j in range(0, steps, 4):
            print("    " + " ".join(f"{x.hex()}," for x in tab[j:j + 4]))
