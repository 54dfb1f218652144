"""The pins are sensitive: plant plausible mistakes in copies of the oracle's
source (on the CPU, in a temporary directory) and check that the same kinds of
checks the real oracle passes catch every one of them.
"""
import ctypes
import json
import os
import subprocess
import tempfile

import numpy as np
import pytest
from numpy.lib.stride_tricks import sliding_window_view

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "wedge.cpp")
GOLD = json.load(open(os.path.join(ROOT, "tests", "golden", "worked_examples.json")))

MUTATIONS = [
    ("no expiry of the leaving location",
     "if (U.front().first == t - w) U.pop_front();", "if (false) U.pop_front();"),
    ("window one element short",
     "if (U.front().first == t - w) U.pop_front();\n      else if (L.front().first == t - w) L.pop_front();",
     "if (U.front().first == t - w + 1) U.pop_front();\n      else if (L.front().first == t - w + 1) L.pop_front();"),
    ("wrong sign in the minimum while-loop", "if (x < L.back().second) L.pop_back();",
     "if (x > L.back().second) L.pop_back();"),
    ("previous location not dropped from U", "        U.pop_back();\n        while (!U.empty()) {",
     "        while (!U.empty()) {"),
    ("inner comparison not counted", "          if (COUNT) ++ncmp;\n          if (x > U.back().second)",
     "          if (x > U.back().second)"),
    ("emission one sample late", "if (t >= w) {  // R4", "if (t >= w + 1) {  // R4"),
    ("naive window one short", "for (int64_t i = j + 1; i < j + w; ++i) {\n      if (a[i] > M)",
     "for (int64_t i = j + 1; i < j + w - 1; ++i) {\n      if (a[i] > M)"),
    ("arg window one short", "for (int64_t i = j + 1; i < j + w; ++i) {\n      if (a[i] > a[im])",
     "for (int64_t i = j + 1; i < j + w - 1; ++i) {\n      if (a[i] > a[im])"),
    ("2-D max taken from the min image", "col[(size_t)r] = rmax[(size_t)(r * oc + c)];",
     "col[(size_t)r] = rmin[(size_t)(r * oc + c)];"),
    ("arg max tie resolved to the right", "if (a[i] > a[im]) im = i;", "if (a[i] >= a[im]) im = i;"),
    ("arg min location off by one", "amn[j] = in;", "amn[j] = in + (in > j ? -1 : 0);"),
    ("deque drops equal values", "while (!U.empty() && a[U.back()] < x) U.pop_back();",
     "while (!U.empty() && a[U.back()] <= x) U.pop_back();"),
    ("deque expires one sample late", "if (L.front() <= i - w) L.pop_front();", "if (L.front() < i - w) L.pop_front();"),
    ("envelope window one short at the right",
     "j1 = i + r > n - 1 ? n - 1 : i + r;", "j1 = i + r > n - 1 ? n - 1 : i + r - (r > 0 ? 1 : 0);"),
    ("envelope not truncated at the left", "const int64_t j0 = i - r < 0 ? 0 : i - r,",
     "const int64_t j0 = i - r < 0 ? (r > 1 ? 1 : 0) : i - r,"),
]


def _compile(src_text, d):
    p = os.path.join(d, "m.cpp")
    with open(p, "w") as f:
        f.write(src_text)
    so = os.path.join(d, "libm.so")
    subprocess.check_call(["g++", "-O1", "-std=c++14", "-shared", "-fPIC", "-o", so, p])
    lib = ctypes.CDLL(so)
    i64, vp = ctypes.c_int64, ctypes.c_void_p
    lib.oracle_wedge.argtypes = [ctypes.c_int, vp, i64, i64, vp, vp, ctypes.POINTER(i64), ctypes.POINTER(i64)]
    lib.oracle_wedge.restype = i64
    lib.oracle_naive.argtypes = [ctypes.c_int, vp, i64, i64, vp, vp]
    lib.oracle_filter2d.argtypes = [ctypes.c_int, vp, i64, i64, i64, i64, i64, vp, vp, i64]
    lib.oracle_argnaive.argtypes = [ctypes.c_int, vp, i64, i64, vp, vp]
    lib.oracle_argdeque.argtypes = [ctypes.c_int, vp, i64, i64, vp, vp]
    lib.oracle_envelope.argtypes = [ctypes.c_int, vp, i64, i64, vp, vp]
    return lib


def _pins_pass(lib):
    """A compact run of the oracle's pins; False as soon as one fails."""
    def call(fn, a, w, count=False):
        k = max(0, a.size - w + 1)
        mx = np.zeros(max(k, 1), np.float64)
        mn = np.zeros(max(k, 1), np.float64)
        c, p = ctypes.c_int64(0), ctypes.c_int64(0)
        if fn == "wedge":
            lib.oracle_wedge(1, a.ctypes.data, a.size, w, mx.ctypes.data, mn.ctypes.data,
                             ctypes.byref(c) if count else None, ctypes.byref(p) if count else None)
        else:
            lib.oracle_naive(1, a.ctypes.data, a.size, w, mx.ctypes.data, mn.ctypes.data)
        return mx[:k], mn[:k], c.value, p.value

    for ex in GOLD["one_d"]:
        a = np.array(ex["a"], np.float64)
        for fn in ("wedge", "naive"):
            mx, mn, c, p = call(fn, a, ex["w"], count=True)
            if mx.tolist() != ex["max"] or mn.tolist() != ex["min"]:
                return False
            if fn == "wedge" and "comparisons" in ex and c != ex["comparisons"]:
                return False
    rng = np.random.default_rng(5)
    for it in range(200):
        n = int(rng.integers(1, 80))
        w = int(rng.integers(1, n + 1))
        a = rng.integers(0, 4, n).astype(np.float64)
        v = sliding_window_view(a, w)
        for fn in ("wedge", "naive"):
            mx, mn, _, _ = call(fn, a, w)
            if not (np.array_equal(mx, v.max(1)) and np.array_equal(mn, v.min(1))):
                return False
    for fn in (lib.oracle_argnaive, lib.oracle_argdeque):
        for ex in GOLD["arg"]:
            a = np.array(ex["a"], np.float64)
            k = a.size - ex["w"] + 1
            imx, imn = np.zeros(k, np.int64), np.zeros(k, np.int64)
            fn(1, a.ctypes.data, a.size, ex["w"], imx.ctypes.data, imn.ctypes.data)
            if imx.tolist() != ex["argmax"] or imn.tolist() != ex["argmin"]:
                return False
        for it in range(100):
            n = int(rng.integers(1, 60))
            w = int(rng.integers(1, n + 1))
            a = rng.integers(0, 4, n).astype(np.float64)
            v = sliding_window_view(a, w)
            j = np.arange(v.shape[0])
            imx, imn = np.zeros(j.size, np.int64), np.zeros(j.size, np.int64)
            fn(1, a.ctypes.data, a.size, w, imx.ctypes.data, imn.ctypes.data)
            if not (np.array_equal(imx, v.argmax(1) + j) and np.array_equal(imn, v.argmin(1) + j)):
                return False
    from scipy.ndimage import maximum_filter1d, minimum_filter1d
    for it in range(100):
        n = int(rng.integers(1, 60))
        r = int(rng.integers(0, n + 2))
        a = rng.integers(0, 9, n).astype(np.float64)
        up, lo = np.zeros(n), np.zeros(n)
        lib.oracle_envelope(1, a.ctypes.data, n, r, up.ctypes.data, lo.ctypes.data)
        if not (np.array_equal(up, maximum_filter1d(a, 2 * r + 1, mode="nearest")) and
                np.array_equal(lo, minimum_filter1d(a, 2 * r + 1, mode="nearest"))):
            return False
    for ex in GOLD["two_d"]:
        a = np.array(ex["a"], np.float64)
        r, c = a.shape
        wr, wc = ex["w_rows"], ex["w_cols"]
        mx = np.zeros((r - wr + 1, c - wc + 1))
        mn = np.zeros_like(mx)
        lib.oracle_filter2d(1, a.ctypes.data, r, c, c, wr, wc, mx.ctypes.data, mn.ctypes.data, c - wc + 1)
        if mx.tolist() != ex["max"] or mn.tolist() != ex["min"]:
            return False
    return True


def test_unmutated_source_passes():
    with tempfile.TemporaryDirectory() as d:
        assert _pins_pass(_compile(open(SRC).read(), d))


@pytest.mark.parametrize("name,old,new", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_planted_mistake_is_caught(name, old, new):
    src = open(SRC).read()
    assert src.count(old) == 1, "mutation anchor not found: " + name
    with tempfile.TemporaryDirectory() as d:
        assert not _pins_pass(_compile(src.replace(old, new), d)), name
