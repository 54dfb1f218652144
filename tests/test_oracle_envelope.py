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


def _scipy_envelope(a, r):
    """The truncated window [max(0, i-r), min(n-1, i+r)] through scipy's
    edge replication (mode='nearest'), independent of the oracle."""
    if a.size == 0:
        return a.copy(), a.copy()
    return maximum_filter1d(a, 2 * r + 1, mode="nearest"), minimum_filter1d(a, 2 * r + 1, mode="nearest")


def test_envelope_batched_hand_example():
    """Two series packed back to back with an empty one between them:
    [3,1,4,1,5] with r = 1, [] with r = 4, [9,2,6] with r = 0."""
    packed = np.array([3, 1, 4, 1, 5, 9, 2, 6], np.float32)
    offs = np.array([0, 5, 5, 8], np.int64)
    up, lo = oracle.envelope_batched(packed, offs, np.array([1, 4, 0], np.int64))
    assert up.tolist() == [3, 4, 4, 5, 5, 9, 2, 6]
    assert lo.tolist() == [1, 1, 1, 1, 1, 9, 2, 6]


@pytest.mark.parametrize("dt", [np.float32, np.float64, np.int32, np.uint16], ids=lambda d: np.dtype(d).name)
def test_envelope_batched_matches_scipy_per_series(dt):
    """A packed buffer with ragged offsets, empty series, r = 0 and r >= n:
    each series' slice equals scipy's nearest-mode filter of that series
    alone, and a brute-force scan of the truncated windows."""
    rng = np.random.default_rng(43)
    for it in range(40):
        S = int(rng.integers(1, 30))
        lens = rng.integers(0, 120, S).astype(np.int64)
        lens[rng.random(S) < 0.2] = 0
        radii = rng.integers(0, 40, S).astype(np.int64)
        radii[rng.random(S) < 0.2] = 0
        big = rng.random(S) < 0.2
        radii[big] = lens[big] + rng.integers(0, 5, int(big.sum()))
        offs = np.zeros(S + 1, np.int64)
        np.cumsum(lens, out=offs[1:])
        packed = rng.integers(0, 30, int(offs[-1])).astype(dt)
        up, lo = oracle.envelope_batched(packed, offs, radii)
        assert up.shape == packed.shape and lo.shape == packed.shape
        for k in range(S):
            s, e, r = int(offs[k]), int(offs[k + 1]), int(radii[k])
            a = packed[s:e]
            su, sl = _scipy_envelope(a, r)
            assert np.array_equal(up[s:e], su) and np.array_equal(lo[s:e], sl), (it, k)
            for i in range(a.size):
                blk = a[max(0, i - r):min(a.size, i + r + 1)]
                assert up[s + i] == blk.max() and lo[s + i] == blk.min(), (it, k, i)
