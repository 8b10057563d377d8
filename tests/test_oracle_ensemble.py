"""Pins of the ensemble-sum oracle (``oracle/ensemble.py``) against what
binary arithmetic fixes: a zero accumulator receives each pixel converted
exactly; integer-valued images add exactly, so every pixel's sum is known in
closed form; zeros change nothing; the placement is checked against the
pixel indices themselves.  CPU only."""
import numpy as np
import pytest

from oracle import ensemble as e


def test_zero_accumulator_receives_exact_conversion():
    rng = np.random.default_rng(1)
    img = rng.standard_normal((5, 7)).astype(np.float32)
    out = e.add_image(np.zeros((9, 11)), img, 3, 2)
    assert np.array_equal(out[2:7, 3:10], img.astype(np.float64))
    assert not out[:2].any() and not out[7:].any() and not out[:, :3].any() and not out[:, 10:].any()


def test_integer_images_add_exactly():
    """Integers below 2^24 are exact in binary32 and their sums below 2^53
    exact in binary64: n overlapping placements give the closed-form count."""
    acc = np.zeros((6, 8))
    imgs, origins = [], []
    for k in range(10):
        imgs.append(np.full((3, 4), float(k + 1), np.float32))
        origins.append((k % 5, k % 4))
    got = e.ensemble_sum((6, 8), imgs, origins)
    want = np.zeros((6, 8))
    for k, (f0, s0) in enumerate(origins):
        want[s0:s0 + 3, f0:f0 + 4] += k + 1
    assert np.array_equal(got, want)


def test_placement_follows_indices():
    """Pixel (c, r) of the image lands on (f0 + c, s0 + r): an image holding
    its own coordinates r * 1000 + c shows up at the right place."""
    r, c = np.meshgrid(np.arange(4), np.arange(6), indexing="ij")
    img = (r * 1000 + c).astype(np.float64)
    out = e.add_image(np.zeros((10, 10)), img, 4, 5)
    rr, cc = np.nonzero(out)
    assert np.array_equal(out[rr, cc], (rr - 5) * 1000 + (cc - 4))
    assert out[5, 4] == 0 and out[8, 9] == 3005


def test_zeros_change_nothing_bitwise():
    rng = np.random.default_rng(2)
    acc = rng.standard_normal((7, 7))
    assert np.array_equal(e.add_image(acc, np.zeros((7, 7), np.float32), 0, 0), acc)


def test_one_rounding_per_addition():
    """acc + x rounds once: 1 + 2^-53 stays 1 (ties to even), 1 + 3 * 2^-53
    rounds up to 1 + 2^-51, checked against the pixel values themselves."""
    acc = np.ones((1, 2))
    img = np.array([[2.0 ** -53, 3 * 2.0 ** -53]])
    out = e.add_image(acc, img, 0, 0)
    assert out[0, 0] == 1.0 and out[0, 1] == 1.0 + 2.0 ** -51


def test_outside_is_refused():
    with pytest.raises(ValueError):
        e.add_image(np.zeros((4, 4)), np.zeros((2, 2)), 3, 0)
