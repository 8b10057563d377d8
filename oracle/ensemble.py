"""Ensemble sums of images, plain numpy (the oracle of ``xrt_add_image``).

TEST INFRASTRUCTURE ONLY: the tests and the benchmark's CPU leg use it; the
product path never imports it, and it shares no code with the HIP library.

Section III of the paper lists a third kernel that adds the results of the
other two into one binary64 image, and its runs reduce the images of many
shots.  The definition written out: for every pixel (c, r) of a region image
placed at (f0, s0), acc[s0 + r, f0 + c] becomes acc[s0 + r, f0 + c] plus the
pixel converted to binary64, one rounding of one binary64 addition.  An
ensemble adds its images one after another in the order given.
"""
from __future__ import annotations

import numpy as np


def add_image(acc: np.ndarray, img: np.ndarray, f0: int, s0: int) -> np.ndarray:
    """A new binary64 array: ``acc`` with ``img`` added at (f0, s0)."""
    acc = np.array(acc, dtype=np.float64, copy=True)
    ns, nf = img.shape
    if f0 < 0 or s0 < 0 or s0 + ns > acc.shape[0] or f0 + nf > acc.shape[1]:
        raise ValueError("image outside the accumulator")
    for r in range(ns):
        for c in range(nf):
            acc[s0 + r, f0 + c] = acc[s0 + r, f0 + c] + np.float64(img[r, c])
    return acc


def ensemble_sum(shape, images, origins) -> np.ndarray:
    """Images added in order into a zero binary64 accumulator of ``shape``."""
    acc = np.zeros(shape, np.float64)
    for img, (f0, s0) in zip(images, origins):
        acc = add_image(acc, img, int(f0), int(s0))
    return acc
