"""Error measures of an image against the oracle's.

* ``max_rel``: max over pixels with ref > 0 of |x - ref| / ref (the headline);
* ``rms_rel``: RMS of the same ratios;
* ``floored``: the same with denominator max(ref, 1e-6 * max(ref));
* ``zeros_ok``: every pixel with ref == 0 is 0 in x as well.
"""
import numpy as np


def compare(x, ref):
    x = np.asarray(x, np.float64)
    ref = np.asarray(ref, np.float64)
    pos = ref > 0
    r = np.abs(x[pos] - ref[pos]) / ref[pos]
    floor = np.maximum(ref, 1e-6 * ref.max()) if ref.size and ref.max() > 0 else np.ones_like(ref)
    rf = np.abs(x - ref) / floor
    return {
        "max_rel": float(r.max()) if r.size else 0.0,
        "rms_rel": float(np.sqrt(np.mean(r * r))) if r.size else 0.0,
        "floored": float(rf.max()) if rf.size else 0.0,
        "zeros_ok": bool(np.all(x[~pos] == 0)),
        "n": int(ref.size),
    }
