"""Pins of the arg max/min oracle (the leftmost location of each window's
maximum and minimum): numpy's argmax/argmin over sliding windows (a library
routine that returns the first occurrence), hand-derived examples, closed
forms, consistency with the value oracle, and the linear-time deque against
the definition."""
import json
import os

import numpy as np
import pytest
from numpy.lib.stride_tricks import sliding_window_view

import oracle
from paper_cs_0610046_amd import synth

GOLD = json.load(open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "worked_examples.json")))
DTS = [np.float32, np.float64, np.int32, np.uint16]


def _np_arg(a, w):
    v = sliding_window_view(a, w)
    j = np.arange(v.shape[0])
    return v.argmax(1) + j, v.argmin(1) + j


@pytest.mark.parametrize("fn", [oracle.argnaive, oracle.argdeque], ids=["naive", "deque"])
def test_hand_examples(fn):
    for ex in GOLD["arg"]:
        a = np.array(ex["a"], np.float64)
        imx, imn = fn(a, ex["w"])
        assert imx.tolist() == ex["argmax"] and imn.tolist() == ex["argmin"], ex["note"]


@pytest.mark.parametrize("dt", DTS, ids=lambda d: np.dtype(d).name)
def test_numpy_first_occurrence_tiny(dt):
    rng = np.random.default_rng(31)
    for _ in range(400):
        n = int(rng.integers(1, 60))
        a = rng.integers(0, 4, n).astype(dt)  # many ties
        for w in range(1, n + 1):
            emx, emn = _np_arg(a, w)
            for fn in (oracle.argnaive, oracle.argdeque):
                imx, imn = fn(a, w)
                assert np.array_equal(imx, emx) and np.array_equal(imn, emn), (fn.__name__, a.tolist(), w)


def test_closed_forms_and_values():
    n = 5000
    up = np.arange(n).astype(np.float64)
    for w in (1, 2, 7, 100, n):
        j = np.arange(n - w + 1)
        for fn in (oracle.argnaive, oracle.argdeque):
            imx, imn = fn(up, w)
            assert np.array_equal(imx, j + w - 1) and np.array_equal(imn, j)
            imx, imn = fn(up[::-1].copy(), w)
            assert np.array_equal(imx, j) and np.array_equal(imn, j + w - 1)
            imx, imn = fn(np.full(n, 3.0), w)
            assert np.array_equal(imx, j) and np.array_equal(imn, j)
    assert oracle.argnaive(np.zeros(3), 4)[0].size == 0


@pytest.mark.parametrize("dt", DTS, ids=lambda d: np.dtype(d).name)
def test_deque_equals_definition_and_values(dt):
    rng = synth.rng_for("tests", 60)
    for kind in ("walk", "ties"):
        n = 20000
        a = synth.small_alphabet(n, 6, dt, rng) if kind == "ties" else \
            synth.random_walk(n, np.float64, rng).astype(dt) if dt in (np.float32, np.float64) else \
            synth.small_alphabet(n, 1000, dt, rng)
        for w in (1, 2, 3, 17, 64, 300):
            imx, imn = oracle.argdeque(a, w)
            nmx, nmn = oracle.argnaive(a, w)
            assert np.array_equal(imx, nmx) and np.array_equal(imn, nmn)
            mx, mn = oracle.wedge(a, w)
            assert np.array_equal(a[imx], mx) and np.array_equal(a[imn], mn)
            j = np.arange(mx.size)
            assert np.all((imx >= j) & (imx < j + w) & (imn >= j) & (imn < j + w))
