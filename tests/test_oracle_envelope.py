"""Pins of the centered-envelope oracle: scipy's maximum/minimum_filter1d
with edge replication ('nearest': a replicated end value is already inside
the truncated window, so the results agree), a hand example, closed forms,
and consistency with the valid-window wedge in the interior."""
import numpy as np
import pytest
from scipy.ndimage import maximum_filter1d, minimum_filter1d

import oracle
from paper_cs_0610046_amd import synth


def test_hand_example():
    a = np.array([3, 1, 4, 1, 5, 9, 2, 6], np.float64)
    up, lo = oracle.envelope(a, 1)
    # windows [0,1] [0,2] [1,3] [2,4] [3,5] [4,6] [5,7] [6,7]
    assert up.tolist() == [3, 4, 4, 5, 9, 9, 9, 6]
    assert lo.tolist() == [1, 1, 1, 1, 1, 2, 2, 2]
    up, lo = oracle.envelope(a, 10)
    assert up.tolist() == [9] * 8 and lo.tolist() == [1] * 8


@pytest.mark.parametrize("dt", [np.float32, np.float64, np.int32, np.uint16], ids=lambda d: np.dtype(d).name)
def test_matches_scipy_nearest(dt):
    rng = np.random.default_rng(41)
    for _ in range(300):
        n = int(rng.integers(1, 200))
        a = rng.integers(0, 50, n).astype(dt)
        for r in (0, 1, 2, 5, int(rng.integers(0, n + 3)), n + 5):
            up, lo = oracle.envelope(a, r)
            assert np.array_equal(up, maximum_filter1d(a, 2 * r + 1, mode="nearest"))
            assert np.array_equal(lo, minimum_filter1d(a, 2 * r + 1, mode="nearest"))


def test_interior_is_the_valid_filter_and_closed_forms():
    rng = synth.rng_for("tests", 61)
    a = synth.random_walk(5000, np.float32, rng)
    for r in (0, 3, 100, 2499):
        up, lo = oracle.envelope(a, r)
        mx, mn = oracle.wedge(a, 2 * r + 1)
        assert np.array_equal(up[r:a.size - r], mx) and np.array_equal(lo[r:a.size - r], mn)
        assert np.all(up >= a) and np.all(lo <= a)
    ramp = np.arange(100, dtype=np.float64)
    up, lo = oracle.envelope(ramp, 7)
    i = np.arange(100)
    assert np.array_equal(up, np.minimum(i + 7, 99)) and np.array_equal(lo, np.maximum(i - 7, 0))
    assert oracle.envelope(np.zeros(0, np.float32), 3)[0].size == 0
