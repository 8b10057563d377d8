"""Arbitrary-precision brute force of the X-ray tracing sum for tiny shots.

TEST INFRASTRUCTURE ONLY: a second, independent statement of the same physics
(paper section II; see ``xro.c`` for the model), used to pin the C oracle.  It
differs from the C oracle on purpose wherever a choice exists:

* 50-digit mpmath arithmetic instead of FP64;
* the lattice factor evaluated from its unreduced definition
  sin^2(pi N h) / sin^2(pi h), not from reduced arguments;
* the polarization factor from explicit angles, 2theta = acos(d . inc);
* the cell matrices built as full matrix products umat * R_phi * U;
* the loops nested in another order (domain, source, then sample point).

The background of an amorphous scatterer is restated the same way
(``background``): stol from the scattering angle instead of |S|/2, the curve
by bisection instead of a scan.

Pure-Python loops: only for a handful of pixels.
"""
from __future__ import annotations

import mpmath as mp

DPS = 50
R_E = mp.mpf("2.8179403262e-15")


def _vec(x):
    return mp.matrix([mp.mpf(float(v)) for v in x])


def _mat(A):
    return mp.matrix([[mp.mpf(float(A[i][j])) for j in range(3)] for i in range(3)])


def _rot(axis, angle):
    u = _vec(axis)
    c, s = mp.cos(angle), mp.sin(angle)
    K = mp.matrix([[0, -u[2], u[1]], [u[2], 0, -u[0]], [-u[1], u[0], 0]])
    return c * mp.eye(3) + s * K + (1 - c) * (u * u.T)


def _dot(a, b):
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]


def _cross(a, b):
    return mp.matrix([a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2],
                      a[0] * b[1] - a[1] * b[0]])


def _lattice_sq(h, N, shape, c):
    if shape == 1:
        f = h - mp.nint(h)
        return N * N * mp.exp(-2 * N * N * f * f / c)
    den = mp.sin(mp.pi * h)
    if den == 0:
        return N * N
    return (mp.sin(mp.pi * N * h) / den) ** 2


def simulate(shot, pixels):
    """Image values (mpf) of the given (i_f, i_s) pixels."""
    with mp.workdps(DPS):
        O = shot.oversample
        fdet, sdet, odet = _vec(shot.fdet), _vec(shot.sdet), _vec(shot.odet)
        p = mp.mpf(float(shot.pixel))
        D = mp.mpf(float(shot.distance))
        dt = mp.mpf(float(shot.layer_dt))
        mu = mp.mpf(float(shot.atten_len))
        K = mp.mpf(float(shot.kahn))
        e = _vec(shot.evec)
        N = [mp.mpf(float(x)) for x in shot.N]
        c = mp.mpf(float(shot.gauss_c))
        U = _mat(shot.U)
        cellT = _mat(shot.cell).T  # columns a, b, c
        hmin = [int(x) for x in shot.hkl_min]
        cnt = shot.F.shape
        mats = []
        for k in range(shot.n_phi):
            phi = mp.mpf(float(shot.phi0)) + k * mp.mpf(float(shot.dphi))
            Rk = _rot(shot.spindle, phi)
            for m in range(shot.n_mos):
                Q = _mat(shot.umats[m]) * Rk * U
                mats.append(Q * cellT)  # columns a', b', c'
        # sample points of every pixel
        def samples(i_f, i_s):
            out = []
            for u in range(O):
                for v in range(O):
                    for t in range(shot.n_layers):
                        Fp = (i_f + (v + mp.mpf(1) / 2) / O) * p - mp.mpf(float(shot.beam_f))
                        Sp = (i_s + (u + mp.mpf(1) / 2) / O) * p - mp.mpf(float(shot.beam_s))
                        r = Fp * fdet + Sp * sdet + (D + t * dt) * odet
                        R = mp.sqrt(_dot(r, r))
                        d = r / R
                        cosrho = _dot(d, odet)
                        dom = p * p * cosrho / (R * R)
                        if dt == 0:
                            cap = mp.mpf(1)
                        else:
                            cap = mp.exp(-t * dt / (mu * cosrho)) - mp.exp(-(t + 1) * dt / (mu * cosrho))
                        out.append((d, dom * cap))
            return out

        res = []
        for (i_f, i_s) in pixels:
            pts = samples(int(i_f), int(i_s))
            total = mp.mpf(0)
            for M in mats:
                for j in range(shot.n_src):
                    inc = _vec(shot.src_dir[j])
                    lam = mp.mpf(float(shot.src_lambda[j]))
                    w = mp.mpf(float(shot.src_weight[j]))
                    ep = e - _dot(e, inc) * inc
                    ep = ep / mp.sqrt(_dot(ep, ep))
                    b = _cross(inc, ep)
                    for (d, geo) in pts:
                        S = (d - inc) / lam
                        two_theta = mp.acos(_dot(d, inc))
                        psi = mp.atan2(_dot(d, b), _dot(d, ep))
                        P = (1 + mp.cos(two_theta) ** 2
                             - K * mp.cos(2 * psi) * mp.sin(two_theta) ** 2) / 2
                        h = [_dot(M[:, i], S) for i in range(3)]
                        L2 = mp.mpf(1)
                        for i in range(3):
                            L2 *= _lattice_sq(h[i], N[i], shot.shape, c)
                        h0 = [int(mp.nint(x)) for x in h]
                        inside = all(hmin[i] <= h0[i] < hmin[i] + cnt[i] for i in range(3))
                        F = (mp.mpf(float(shot.F[h0[0] - hmin[0], h0[1] - hmin[1], h0[2] - hmin[2]]))
                             if inside else mp.mpf(float(shot.F_default)))
                        total += w * P * geo * F * F * L2
            norm = (R_E ** 2 * mp.mpf(float(shot.fluence)) * mp.mpf(float(shot.scale))
                    / (O * O * shot.n_phi * shot.n_mos))
            res.append(norm * total)
        return res


def _bg_curve(stol, F, x):
    """Piecewise-linear interpolation by bisection over the knots (the C oracle
    scans them), constant beyond the ends."""
    import bisect
    xs = [mp.mpf(float(v)) for v in stol]
    if x <= xs[0]:
        return mp.mpf(float(F[0]))
    if x >= xs[-1]:
        return mp.mpf(float(F[-1]))
    k = bisect.bisect_right(xs, x) - 1
    a, b = mp.mpf(float(F[k])), mp.mpf(float(F[k + 1]))
    return (a * (xs[k + 1] - x) + b * (x - xs[k])) / (xs[k + 1] - xs[k])


def background(shot, bg, pixels):
    """Background of an amorphous scatterer (mpf) at the given pixels, from
    angles: stol = sin(theta)/lambda with 2 theta = acos(d . inc), and the
    polarization from explicit 2 theta and psi; loops source-outermost."""
    with mp.workdps(DPS):
        O = shot.oversample
        fdet, sdet, odet = _vec(shot.fdet), _vec(shot.sdet), _vec(shot.odet)
        p = mp.mpf(float(shot.pixel))
        D = mp.mpf(float(shot.distance))
        dt = mp.mpf(float(shot.layer_dt))
        mu = mp.mpf(float(shot.atten_len))
        K = mp.mpf(float(shot.kahn))
        e = _vec(shot.evec)
        res = []
        for (i_f, i_s) in pixels:
            total = mp.mpf(0)
            for j in range(shot.n_src):
                inc = _vec(shot.src_dir[j])
                lam = mp.mpf(float(shot.src_lambda[j]))
                w = mp.mpf(float(shot.src_weight[j]))
                ep = e - _dot(e, inc) * inc
                ep = ep / mp.sqrt(_dot(ep, ep))
                b = _cross(inc, ep)
                for t in range(shot.n_layers):
                    for u in range(O):
                        for v in range(O):
                            Fp = (int(i_f) + (v + mp.mpf(1) / 2) / O) * p - mp.mpf(float(shot.beam_f))
                            Sp = (int(i_s) + (u + mp.mpf(1) / 2) / O) * p - mp.mpf(float(shot.beam_s))
                            r = Fp * fdet + Sp * sdet + (D + t * dt) * odet
                            R = mp.sqrt(_dot(r, r))
                            d = r / R
                            cosrho = _dot(d, odet)
                            dom = p * p * cosrho / (R * R)
                            if dt == 0:
                                cap = mp.mpf(1)
                            else:
                                cap = (mp.exp(-t * dt / (mu * cosrho))
                                       - mp.exp(-(t + 1) * dt / (mu * cosrho)))
                            two_theta = mp.acos(_dot(d, inc))
                            psi = mp.atan2(_dot(d, b), _dot(d, ep))
                            P = (1 + mp.cos(two_theta) ** 2
                                 - K * mp.cos(2 * psi) * mp.sin(two_theta) ** 2) / 2
                            Fb = _bg_curve(bg.stol, bg.F, mp.sin(two_theta / 2) / lam)
                            total += w * P * dom * cap * Fb * Fb
            res.append(R_E ** 2 * mp.mpf(float(shot.fluence)) * mp.mpf(float(bg.molecules))
                       / (O * O) * total)
        return res


def term_condition(shot, pixels):
    """Per pixel, an estimate of |d ln I| caused by the FP64 rounding of h:
    the sum over terms of term * sum_i |d ln L2_i / dh_i| * dh_i, divided by
    the pixel sum, with dh_i = |a'_i| eps / lambda (one rounding of d - inc,
    which cancels in its z part) + 4 ulp(h_i).  Used to size tolerances of
    comparisons whose pixels hold few, ill-conditioned terms."""
    import math
    with mp.workdps(30):
        out = []
        U = _mat(shot.U)
        cellT = _mat(shot.cell).T
        for (i_f, i_s) in pixels:
            tot, sens = mp.mpf(0), mp.mpf(0)
            O = shot.oversample
            for k in range(shot.n_phi):
                Rk = _rot(shot.spindle, mp.mpf(float(shot.phi0)) + k * mp.mpf(float(shot.dphi)))
                for m in range(shot.n_mos):
                    M = _mat(shot.umats[m]) * Rk * U * cellT
                    for j in range(shot.n_src):
                        inc = _vec(shot.src_dir[j])
                        lam = mp.mpf(float(shot.src_lambda[j]))
                        for u in range(O):
                            for v in range(O):
                                for t in range(shot.n_layers):
                                    Fp = (i_f + (v + 0.5) / O) * shot.pixel - shot.beam_f
                                    Sp = (i_s + (u + 0.5) / O) * shot.pixel - shot.beam_s
                                    r = (Fp * _vec(shot.fdet) + Sp * _vec(shot.sdet)
                                         + (shot.distance + t * shot.layer_dt) * _vec(shot.odet))
                                    d = r / mp.sqrt(_dot(r, r))
                                    S = (d - inc) / lam
                                    term, s = mp.mpf(1), mp.mpf(0)
                                    for i in range(3):
                                        h = _dot(M[:, i], S)
                                        Ni = mp.mpf(float(shot.N[i]))
                                        term *= _lattice_sq(h, Ni, shot.shape, shot.gauss_c)
                                        dl = mp.diff(lambda x: mp.log(_lattice_sq(x, Ni, shot.shape, shot.gauss_c)), h)
                                        dh = (mp.norm(M[:, i]) * 2.0 ** -52 / lam
                                              + 4 * math.ulp(float(h)))
                                        s += abs(dl) * dh
                                    tot += term
                                    sens += term * s
            out.append(float(sens / tot) if tot > 0 else 0.0)
        return out
