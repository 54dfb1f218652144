"""The other exact filters the paper reviews, as cross-checks of the
definition (and so of the oracle): van Herk / Gil-Werman and Gil-Kimmel
(Related Work) and the two-comparison w = 3 filter (the lower-bound
section's proposition).  Values must equal the definition; comparison
counts must meet the bounds the paper states for each."""
import math

import numpy as np
import pytest
from numpy.lib.stride_tricks import sliding_window_view

import oracle
from paper_cs_0610046_amd import synth

DTS = [np.float32, np.float64, np.int32, np.uint16]


@pytest.mark.parametrize("dt", DTS, ids=lambda d: np.dtype(d).name)
def test_values_equal_definition(dt):
    rng = np.random.default_rng(51)
    for _ in range(300):
        n = int(rng.integers(1, 70))
        a = rng.integers(0, 5, n).astype(dt)
        for w in range(1, n + 2):
            emx, emn = oracle.naive(a, w)
            for fn in (oracle.vhgw, oracle.gil_kimmel):
                mx, mn, _ = fn(a, w)
                assert np.array_equal(mx, emx) and np.array_equal(mn, emn), (fn.__name__, a.tolist(), w)
        mx, mn, _ = oracle.minmax3(a)
        emx, emn = oracle.naive(a, 3)
        assert np.array_equal(mx, emx) and np.array_equal(mn, emn)


def test_larger_inputs_equal_wedge():
    rng = synth.rng_for("tests", 52)
    a = synth.random_walk(200000, np.float64, rng)
    for w in (2, 3, 10, 97, 1000, 4096):
        emx, emn = oracle.wedge(a, w)
        for fn in (oracle.vhgw, oracle.gil_kimmel):
            mx, mn, _ = fn(a, w)
            assert np.array_equal(mx, emx) and np.array_equal(mn, emn)


def test_vhgw_count_is_6_minus_8_over_w():
    """n = k*w: per direction, k blocks of (w-1) prefix + (w-2) suffix
    comparisons, and one per window not starting a block: 3w-4 per block as
    the paper counts, i.e. 6 - 8/w per element for max and min together
    (less the k - 1 windows a series of k blocks does not have)."""
    rng = np.random.default_rng(53)
    for w in (2, 3, 5, 16, 100):
        for k in (1, 2, 7, 40):
            n = k * w
            a = rng.standard_normal(n)
            _, _, c = oracle.vhgw(a, w)
            per_dir = k * (2 * w - 3) + (n - w + 1 - k)
            assert c == 2 * per_dir
            assert c <= n * (6 - 8 / w) + 1e-9


def test_gil_kimmel_count_bound():
    """Per block and direction: about 1.5 w comparisons for the prefixes and
    suffixes plus a binary search of ceil(log2 w): the paper's
    3 + 2 log(w)/w per element for max and min, up to O(1/w)."""
    rng = np.random.default_rng(54)
    for w in (4, 8, 16, 64, 256, 1024):
        n = 200 * w
        for kind in ("noise", "ramp", "ties"):
            a = rng.standard_normal(n) if kind == "noise" else (np.arange(n, dtype=np.float64) if kind == "ramp"
                                                                 else rng.integers(0, 3, n).astype(np.float64))
            _, _, c = oracle.gil_kimmel(a, w)
            assert c <= n * (3 + (2 * math.log2(w) + 6) / w), (w, kind, c / n)
            _, _, cv = oracle.vhgw(a, w)
            if w >= 8:
                assert c < cv  # fewer than van Herk / Gil-Werman


def test_minmax3_two_comparisons():
    rng = np.random.default_rng(55)
    for n in (3, 4, 10, 1001):
        a = rng.integers(0, 4, n).astype(np.float64)
        _, _, c = oracle.minmax3(a)
        assert c == 2 * n - 3  # one for the first pair, then two per sample
    assert oracle.minmax3(np.zeros(2))[2] == 0
