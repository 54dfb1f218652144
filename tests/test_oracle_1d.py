"""Pins for the 1-D CPU oracle (no GPU).

The oracle is pinned to things other than itself:
* hand-derived worked examples (tests/golden/worked_examples.json),
* numpy's sliding_window_view max/min and scipy's maximum_filter1d /
  minimum_filter1d (library routines for the same definition),
* brute force (the definition, Section 1) on tiny inputs, against the wedge
  (Section 4, Algorithm 1),
* closed forms (w = 1, w = n, ramps, constants, a sine of period p with w >= p),
* invariants (window bounds attained; wedge size <= w + 1, the memory
  proposition of Section 4),
* the comparison bounds of Section 4 (at most 3 per element; exactly one per
  element on strictly monotone input).
"""
import json
import os

import numpy as np
import pytest
from numpy.lib.stride_tricks import sliding_window_view

import oracle
from paper_cs_0610046_amd import synth

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "worked_examples.json")))
DTS = [np.float32, np.float64, np.int32, np.uint16]


def lib_maxmin(a, w):
    """numpy library routine for the definition."""
    if a.size < w:
        return a[:0].copy(), a[:0].copy()
    v = sliding_window_view(a, w)
    return v.max(axis=1), v.min(axis=1)


@pytest.mark.parametrize("ex", GOLD["one_d"], ids=lambda e: "n%d_w%d" % (len(e["a"]), e["w"]))
@pytest.mark.parametrize("dt", [np.float32, np.float64, np.int32])
def test_worked_examples(ex, dt):
    a = np.array(ex["a"], dt)
    for fn in (oracle.naive, oracle.wedge):
        mx, mn = fn(a, ex["w"])
        assert mx.tolist() == ex["max"] and mn.tolist() == ex["min"], fn.__name__
    mx, mn, c, peak = oracle.wedge(a, ex["w"], count=True)
    if "comparisons" in ex:
        assert c == ex["comparisons"]
    if "peak_wedge" in ex:
        assert peak == ex["peak_wedge"]


def test_worked_stream():
    for ex in GOLD["stream"]:
        s = oracle.Stream(np.float64, ex["w"])
        for chunk, emx, emn in zip(ex["chunks"], ex["max"], ex["min"]):
            mx, mn = s.push(np.array(chunk, np.float64))
            assert mx.tolist() == emx and mn.tolist() == emn


def test_naive_matches_numpy_library():
    rng = synth.rng_for("tests", 1)
    for it in range(300):
        dt = DTS[it % 4]
        n = int(rng.integers(0, 200))
        w = int(rng.integers(1, n + 4))
        a = synth.small_alphabet(n, 1000, dt, rng) if it % 3 else synth.small_alphabet(n, 3, dt, rng)
        mx, mn = oracle.naive(a, w)
        lmx, lmn = lib_maxmin(a, w)
        assert np.array_equal(mx, lmx) and np.array_equal(mn, lmn)


def test_naive_matches_scipy_library():
    ndi = pytest.importorskip("scipy.ndimage")
    # scipy centres its window: with origin o the output at i covers
    # [i - w//2 - o, i - w//2 - o + w); the 0-based valid window [j, j+w)
    # is output index j + w//2 + o with o = -(w//2) -> index j.
    a = np.array([3, 1, 4, 1, 5, 9, 2, 6], np.float64)
    w = 3
    o = -(w // 2)
    full = ndi.maximum_filter1d(a, w, origin=o, mode="nearest")
    assert full[:a.size - w + 1].tolist() == [4, 4, 5, 9, 9, 9]  # the hand example
    rng = synth.rng_for("tests", 2)
    for it in range(100):
        n = int(rng.integers(1, 300))
        w = int(rng.integers(1, n + 1))
        a = rng.standard_normal(n)
        o = -(w // 2)
        smx = ndi.maximum_filter1d(a, w, origin=o, mode="nearest")[:n - w + 1]
        smn = ndi.minimum_filter1d(a, w, origin=o, mode="nearest")[:n - w + 1]
        mx, mn = oracle.naive(a, w)
        assert np.array_equal(mx, smx) and np.array_equal(mn, smn)


@pytest.mark.parametrize("dt", DTS)
def test_wedge_equals_brute_force(dt):
    rng = synth.rng_for("tests", 3)
    for it in range(1500):
        n = int(rng.integers(0, 120))
        w = int(rng.integers(1, n + 4))
        k = [2, 3, 5, 50, 60000][it % 5]
        a = synth.small_alphabet(n, k, dt, rng)
        if it % 7 == 0:
            a = np.sort(a)
        if it % 11 == 0:
            a = np.sort(a)[::-1].copy()
        mx, mn = oracle.wedge(a, w)
        bmx, bmn = oracle.naive(a, w)
        assert np.array_equal(mx, bmx), (n, w, a.tolist())
        assert np.array_equal(mn, bmn), (n, w, a.tolist())


def test_wedge_larger_random_walks():
    rng = synth.rng_for("tests", 4)
    for n, w in [(5000, 1), (5000, 2), (5000, 17), (5000, 64), (5000, 999), (5000, 5000), (3000, 4000)]:
        a = synth.random_walk(n, np.float32, rng)
        mx, mn = oracle.wedge(a, w)
        lmx, lmn = lib_maxmin(a, w)
        assert np.array_equal(mx, lmx) and np.array_equal(mn, lmn)


def test_closed_forms():
    rng = synth.rng_for("tests", 5)
    a = synth.random_walk(777, np.float64, rng)
    # w = 1: identity
    mx, mn = oracle.wedge(a, 1)
    assert np.array_equal(mx, a) and np.array_equal(mn, a)
    # w = n: one window, the global extrema
    mx, mn = oracle.wedge(a, a.size)
    assert mx.tolist() == [a.max()] and mn.tolist() == [a.min()]
    # w > n: nothing
    mx, mn = oracle.wedge(a, a.size + 1)
    assert mx.size == 0 and mn.size == 0
    # strictly increasing ramp: max is the window's last element, min its first
    r = synth.ramp_f32(1000)
    for w in (2, 7, 64, 1000):
        mx, mn = oracle.wedge(r, w)
        assert np.array_equal(mx, r[w - 1:]) and np.array_equal(mn, r[:r.size - w + 1])
        d = r[::-1].copy()
        mx, mn = oracle.wedge(d, w)
        assert np.array_equal(mx, d[:d.size - w + 1]) and np.array_equal(mn, d[w - 1:])
    # constant series
    c = np.full(100, 7, np.int32)
    mx, mn = oracle.wedge(c, 13)
    assert np.all(mx == 7) and np.all(mn == 7) and mx.size == 88
    # sine of period p: every window of width >= p attains the global extrema
    p = 100
    s = synth.sine(2000, period=p)
    mx, mn = oracle.wedge(s, p + 1)
    assert np.all(mx == s.max()) and np.all(mn == s.min())


def test_window_invariants():
    rng = synth.rng_for("tests", 6)
    for it in range(50):
        n = int(rng.integers(1, 400))
        w = int(rng.integers(1, n + 1))
        a = rng.standard_normal(n)
        mx, mn = oracle.wedge(a, w)
        v = sliding_window_view(a, w)
        assert np.all(mx[:, None] >= v) and np.all(mn[:, None] <= v)
        assert np.all(np.any(v == mx[:, None], axis=1))
        assert np.all(np.any(v == mn[:, None], axis=1))


def test_comparison_bound_and_wedge_size():
    """At most 3 comparisons per element (Section 4, the proposition bounding
    Algorithm 1 by 3n); size(U)+size(L) <= w+1 (the memory proposition)."""
    rng = synth.rng_for("tests", 7)
    for it in range(400):
        n = int(rng.integers(0, 300))
        w = int(rng.integers(1, n + 3))
        kind = it % 4
        if kind == 0:
            a = rng.standard_normal(n)
        elif kind == 1:
            a = synth.small_alphabet(n, 3, np.float64, rng)
        elif kind == 2:
            a = synth.piecewise_monotone(n, np.float64, rng, mean_run=5)
        else:
            a = np.cumsum(rng.standard_normal(n))
        mx, mn, c, peak = oracle.wedge(a, w, count=True)
        assert c <= 3 * n
        assert c <= 3 * max(n - 1, 0)  # tighter: the first element is never compared
        if n:
            assert peak <= w + 1


def test_strictly_monotone_costs_one_comparison_per_element():
    """Strictly monotone input: the inner while-loops never make a comparison
    that is true, so the cost is within the paper's 2 per element; in this
    update order it is exactly one per new element."""
    for n, w in [(1000, 3), (1000, 64), (5000, 999)]:
        up = synth.ramp_f32(n)
        for a in (up, up[::-1].copy()):
            mx, mn, c, _ = oracle.wedge(a, w, count=True)
            assert c == n - 1
            assert c <= 2 * n


def test_non_strict_monotone_reading():
    """Reading taken of the monotone-input proposition: it holds for strictly
    monotone data; with plateaus (non-decreasing, equal neighbours) the equal
    values go to U and are popped later by true comparisons, so the count can
    exceed 2 per element (it stays within 3)."""
    a = np.repeat(np.arange(2000, dtype=np.float64), 5)
    mx, mn, c, _ = oracle.wedge(a, 50, count=True)
    assert c > 2 * (a.size - 1)
    assert c <= 3 * (a.size - 1)


def test_iid_count_near_paper_regime():
    """On i.i.d. noise the count per element stays below 3 and approaches 3
    as w grows (the worst case of Table 1)."""
    rng = synth.rng_for("tests", 8)
    a = rng.random(200000)
    prev = 0.0
    for w in (3, 16, 64, 1024):
        _, _, c, _ = oracle.wedge(a, w, count=True)
        r = c / a.size
        assert r <= 3.0 and r >= prev - 1e-3
        prev = r
    assert prev > 2.9


@pytest.mark.parametrize("dt", DTS)
def test_stream_chunking_invariance(dt):
    rng = synth.rng_for("tests", 9)
    for it in range(60):
        n = int(rng.integers(0, 3000))
        w = int(rng.integers(1, 700))
        a = synth.small_alphabet(n, 40, dt, rng)
        ref_mx, ref_mn = oracle.wedge(a, w)
        s = oracle.Stream(dt, w)
        outs_mx, outs_mn = [], []
        pos = 0
        while pos < n:
            m = int(rng.integers(0, 300))
            mx, mn = s.push(a[pos:pos + m])
            outs_mx.append(mx)
            outs_mn.append(mn)
            pos += m
        got_mx = np.concatenate(outs_mx) if outs_mx else a[:0]
        got_mn = np.concatenate(outs_mn) if outs_mn else a[:0]
        assert np.array_equal(got_mx, ref_mx) and np.array_equal(got_mn, ref_mn)
        st = s.stats()
        assert st["t"] == n
        s.close()


@pytest.mark.parametrize("dt", DTS)
def test_stream_export_resume_round_trip(dt):
    """A stream exported at any point (t, last min(t, w-1) samples) and
    resumed in a fresh wedge continues exactly as the uninterrupted stream:
    the concatenated outputs equal the one-shot filter (the definition's
    windows each depend on their own w samples only)."""
    rng = synth.rng_for("tests", 12)
    for it in range(60):
        n = int(rng.integers(0, 2500))
        w = int(rng.integers(1, 600))
        a = synth.small_alphabet(n, 30, dt, rng)
        ref_mx, ref_mn = oracle.wedge(a, w)
        s = oracle.Stream(dt, w)
        outs_mx, outs_mn = [], []
        pos = 0
        while pos < n:
            m = int(rng.integers(0, 250))
            mx, mn = s.push(a[pos:pos + m])
            outs_mx.append(mx)
            outs_mn.append(mn)
            pos += m
            if rng.random() < 0.4:  # checkpoint and resume
                t, carry = s.export()
                assert t == min(pos, n)
                assert np.array_equal(carry, a[max(0, t - (w - 1)):t])
                s.close()
                s = oracle.Stream.resume(dt, w, t, carry)
        got_mx = np.concatenate(outs_mx) if outs_mx else a[:0]
        got_mn = np.concatenate(outs_mn) if outs_mn else a[:0]
        assert np.array_equal(got_mx, ref_mx) and np.array_equal(got_mn, ref_mn)
        s.close()
    with pytest.raises(ValueError):
        oracle.Stream.resume(dt, 5, 10, np.zeros(3, dt))  # min(10, 4) = 4 samples needed


def test_stream_push_counts():
    """n_out of a push = max(0, t+m-w+1) - max(0, t-w+1)."""
    s = oracle.Stream(np.float32, 10)
    t = 0
    rng = synth.rng_for("tests", 10)
    for m in [0, 3, 4, 1, 1, 1, 20, 0, 7]:
        mx, _ = s.push(rng.random(m, dtype=np.float32))
        assert mx.size == max(0, t + m - 10 + 1) - max(0, t - 10 + 1)
        t += m


def test_bad_arguments():
    with pytest.raises(ValueError):
        oracle.wedge(np.zeros(4, np.float32), 0)
    with pytest.raises(TypeError):
        oracle.wedge(np.zeros(4, np.int8), 2)
