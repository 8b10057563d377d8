"""Error measures of an image against the oracle's.

* ``max_rel``: max over resolved pixels (ref >= tiny, ref > 0) of
  |x - ref| / ref (the headline);
* ``rms_rel``: RMS of the same ratios;
* ``floored``: the same with denominator max(ref, 1e-6 * max(ref));
* ``zeros_ok``: every pixel with ref == 0 is 0 in x as well.

``tiny`` (default 0: every pixel with ref > 0 counts) is for outputs whose
small values lie in the subnormal binary64 range, where a number carries no
relative precision in either implementation (the Gaussian shape's tails reach
it: its exponent falls to about -950 at N = 20 and -3800 at N = 40).  With
``tiny = 2^-1022`` (the smallest normal binary64) pixels below it are held
to an absolute |x - ref| <= tol * tiny instead (``sub_abs``, reported as a
multiple of tiny), and ``zeros_ok`` asks that a zero on either side is
matched by a value below tiny on the other.
"""
import numpy as np

DBL_MIN = float(np.finfo(np.float64).tiny)


def compare(x, ref, tiny=0.0):
    x = np.asarray(x, np.float64)
    ref = np.asarray(ref, np.float64)
    pos = (ref >= tiny) & (ref > 0)
    r = np.abs(x[pos] - ref[pos]) / ref[pos]
    floor = np.maximum(ref, 1e-6 * ref.max()) if ref.size and ref.max() > 0 else np.ones_like(ref)
    rf = np.abs(x - ref) / floor
    out = {
        "max_rel": float(r.max()) if r.size else 0.0,
        "rms_rel": float(np.sqrt(np.mean(r * r))) if r.size else 0.0,
        "floored": float(rf.max()) if rf.size else 0.0,
        "n": int(ref.size),
        "n_resolved": int(pos.sum()),
    }
    if tiny > 0:
        sub = ~pos
        out["sub_abs"] = float(np.max(np.abs(x[sub] - ref[sub])) / tiny) if sub.any() else 0.0
        out["zeros_ok"] = bool(np.all(np.abs(x[ref == 0]) < tiny) and np.all(ref[x == 0] < tiny))
    else:
        out["zeros_ok"] = bool(np.all(x[ref <= 0] == 0))
    return out
