"""Minimax fits of sin(pi x) used by the device kernels.

sin(pi x) = x * P(x^2) on |x| <= 1/2, with P minimising the maximum relative
error of x P(x^2) over the interval (equivalently of P(y) against
sin(pi sqrt y)/sqrt y on 0 <= y <= 1/4).  The fit is the Remez exchange
algorithm (Remez 1934; see e.g. Muller, "Elementary Functions", ch. 3) run in
50-digit mpmath, then rounded to the storage precision and re-checked on a
dense grid.  Run as a script to print the coefficient tables that
``xrt_math.h`` carries.
"""
from __future__ import annotations

import sys

import mpmath as mp

mp.mp.dps = 50
Y1 = mp.mpf(1) / 4


def target(y):
    if y == 0:
        return +mp.pi
    r = mp.sqrt(y)
    return mp.sin(mp.pi * r) / r


def remez(deg: int, iters: int = 30):
    """Coefficients c_0..c_deg of the relative-minimax P on [0, 1/4]."""
    n = deg + 2
    # Chebyshev extrema as the initial reference
    xs = [Y1 * (1 - mp.cos(mp.pi * i / (n - 1))) / 2 for i in range(n)]
    E = mp.mpf(0)
    for _ in range(iters):
        A = mp.matrix(n, n)
        b = mp.matrix(n, 1)
        for i, x in enumerate(xs):
            t = target(x)
            for j in range(deg + 1):
                A[i, j] = x ** j
            A[i, deg + 1] = (-1) ** i * t
            b[i] = t
        sol = mp.lu_solve(A, b)
        c = [sol[j] for j in range(deg + 1)]
        E = sol[deg + 1]

        def err(y):
            return (mp.polyval(c[::-1], y) - target(y)) / target(y)
        # new reference: extrema of the error between sign changes
        grid = [Y1 * i / 4000 for i in range(4001)]
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
            # keep the n largest alternating extrema, in order
            while len(ext) > n:
                a0, a1 = abs(err(ext[0])), abs(err(ext[-1]))
                ext.pop(0 if a0 < a1 else -1)
            xs = ext
    return c, abs(E)


def max_rel_err(coeffs, to_float, n=200001):
    """Max relative error of x P(x^2), coefficients rounded by to_float and
    evaluated by Horner in exact arithmetic (isolates the fit + rounding)."""
    cs = [mp.mpf(to_float(float(c))) for c in coeffs]
    worst = mp.mpf(0)
    for i in range(1, n):
        x = mp.mpf(i) / (2 * (n - 1))
        y = x * x
        p = mp.polyval(cs[::-1], y)
        worst = max(worst, abs(x * p / mp.sin(mp.pi * x) - 1))
    return worst


def main():
    import numpy as np
    for name, deg, rnd in (("SINPI_F64", 7, float), ("SINPI_F32", 4, lambda v: float(np.float32(v)))):
        c, E = remez(deg)
        worst = max_rel_err(c, rnd, 20001)
        print(f"// {name}: degree {deg} in x^2, Remez level {mp.nstr(E, 3)}, "
              f"max rel err after rounding {mp.nstr(worst, 3)}")
        suffix = "" if name.endswith("64") else "f"
        for j, v in enumerate(c):
            print(f"    {rnd(float(v))!r}{suffix},   // c{j}")
    return 0


if __name__ == "__main__":
    sys.exit(main())
