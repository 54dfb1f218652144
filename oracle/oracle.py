"""ctypes wrapper of the CPU oracle (``oracle/wedge.cpp``) -- test infrastructure.

Built with ``g++ -O2`` (the optimisation level the paper's experiments used,
Section 5) into ``oracle/_build/liboracle.so``.  Nothing here touches a GPU.
"""
import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "wedge.cpp")
_OUT_DIR = os.path.join(_HERE, "_build")
_LIB_PATH = os.path.join(_OUT_DIR, "liboracle.so")

# dtype codes understood by wedge.cpp
DTYPES = {np.dtype(np.float32): 0, np.dtype(np.float64): 1,
          np.dtype(np.int32): 2, np.dtype(np.uint16): 3}

_lock = threading.Lock()
_lib = None

_i64 = ctypes.c_int64
_vp = ctypes.c_void_p
_i64p = ctypes.POINTER(ctypes.c_int64)


def build(force=True):
    """Compile the oracle with g++ (-O2, no fast-math)."""
    os.makedirs(_OUT_DIR, exist_ok=True)
    if not force and os.path.exists(_LIB_PATH) and \
            os.path.getmtime(_LIB_PATH) >= os.path.getmtime(_SRC):
        return _LIB_PATH
    tmp = _LIB_PATH + ".tmp%d" % os.getpid()
    subprocess.check_call(["g++", "-O2", "-std=c++14", "-shared", "-fPIC",
                           "-Wall", "-o", tmp, _SRC])
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def load():
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        build(force=False)
        lib = ctypes.CDLL(_LIB_PATH)
        lib.oracle_naive.argtypes = [ctypes.c_int, _vp, _i64, _i64, _vp, _vp]
        lib.oracle_naive.restype = ctypes.c_int
        lib.oracle_wedge.argtypes = [ctypes.c_int, _vp, _i64, _i64, _vp, _vp, _i64p, _i64p]
        lib.oracle_wedge.restype = _i64
        lib.oracle_stream_create.argtypes = [ctypes.c_int, _i64]
        lib.oracle_stream_create.restype = _vp
        lib.oracle_stream_push.argtypes = [_vp, _vp, _i64, _vp, _vp]
        lib.oracle_stream_push.restype = _i64
        lib.oracle_stream_stats.argtypes = [_vp, _i64p, _i64p, _i64p]
        lib.oracle_stream_stats.restype = ctypes.c_int
        lib.oracle_stream_destroy.argtypes = [_vp]
        lib.oracle_stream_destroy.restype = None
        for f in (lib.oracle_filter2d, lib.oracle_naive2d):
            f.argtypes = [ctypes.c_int, _vp, _i64, _i64, _i64, _i64, _i64, _vp, _vp, _i64]
            f.restype = ctypes.c_int
        for f in (lib.oracle_vhgw, lib.oracle_gil_kimmel):
            f.argtypes = [ctypes.c_int, _vp, _i64, _i64, _vp, _vp]
            f.restype = _i64
        lib.oracle_minmax3.argtypes = [ctypes.c_int, _vp, _i64, _vp, _vp]
        lib.oracle_minmax3.restype = _i64
        lib.oracle_envelope.argtypes = [ctypes.c_int, _vp, _i64, _i64, _vp, _vp]
        lib.oracle_envelope.restype = ctypes.c_int
        for f in (lib.oracle_argnaive, lib.oracle_argdeque):
            f.argtypes = [ctypes.c_int, _vp, _i64, _i64, _vp, _vp]
            f.restype = ctypes.c_int
        _lib = lib
        return lib


def _code(a):
    try:
        return DTYPES[a.dtype]
    except KeyError:
        raise TypeError("oracle: unsupported dtype %s" % a.dtype)


def _ptr(a):
    return ctypes.c_void_p(a.ctypes.data) if a.size else ctypes.c_void_p(0)


def n_out(n, w):
    """Number of valid windows: max(0, n - w + 1)."""
    return max(0, int(n) - int(w) + 1)


def naive(a, w):
    """Definition of the filter: scan every window (O(n*w))."""
    a = np.ascontiguousarray(a)
    k = n_out(a.size, w)
    mx = np.empty(k, a.dtype)
    mn = np.empty(k, a.dtype)
    if load().oracle_naive(_code(a), _ptr(a), a.size, int(w), _ptr(mx), _ptr(mn)) != 0:
        raise ValueError("oracle_naive: bad arguments")
    return mx, mn


def wedge(a, w, count=False):
    """Algorithm 1 over the whole series.

    Returns ``(max, min)``, or ``(max, min, comparisons, peak_wedge_size)``
    when ``count`` is true.
    """
    a = np.ascontiguousarray(a)
    if int(w) < 1:
        raise ValueError("w must be >= 1")
    k = n_out(a.size, w)
    mx = np.empty(k, a.dtype)
    mn = np.empty(k, a.dtype)
    c = ctypes.c_int64(0)
    p = ctypes.c_int64(0)
    got = load().oracle_wedge(_code(a), _ptr(a), a.size, int(w), _ptr(mx), _ptr(mn),
                              ctypes.byref(c) if count else None,
                              ctypes.byref(p) if count else None)
    if got != k:
        raise RuntimeError("oracle_wedge returned %d windows, expected %d" % (got, k))
    if count:
        return mx, mn, c.value, p.value
    return mx, mn


def _arg(fn, a, w):
    a = np.ascontiguousarray(a)
    if int(w) < 1:
        raise ValueError("w must be >= 1")
    k = n_out(a.size, w)
    imx = np.empty(k, np.int64)
    imn = np.empty(k, np.int64)
    if fn(_code(a), _ptr(a), a.size, int(w), _ptr(imx), _ptr(imn)) != 0:
        raise ValueError("bad arguments")
    return imx, imn


def _cross(fn, a, w):
    a = np.ascontiguousarray(a)
    k = n_out(a.size, w)
    mx = np.empty(k, a.dtype)
    mn = np.empty(k, a.dtype)
    c = fn(a, mx, mn)
    if c < 0:
        raise ValueError("bad arguments")
    return mx, mn, int(c)


def vhgw(a, w):
    """van Herk / Gil-Werman (Related Work): ``(max, min, comparisons)``."""
    return _cross(lambda a, x, y: load().oracle_vhgw(_code(a), _ptr(a), a.size, int(w), _ptr(x), _ptr(y)), a, w)


def gil_kimmel(a, w):
    """Gil-Kimmel (Related Work): ``(max, min, comparisons)``."""
    return _cross(lambda a, x, y: load().oracle_gil_kimmel(_code(a), _ptr(a), a.size, int(w), _ptr(x), _ptr(y)), a, w)


def minmax3(a):
    """The two-comparison w = 3 filter (lower-bound section):
    ``(max, min, comparisons)``."""
    return _cross(lambda a, x, y: load().oracle_minmax3(_code(a), _ptr(a), a.size, _ptr(x), _ptr(y)), a, 3)


def envelope(a, r):
    """Centered envelope of radius r (definition): upper[i] / lower[i] = max /
    min of a over [max(0, i-r), min(n-1, i+r)]."""
    a = np.ascontiguousarray(a)
    if int(r) < 0:
        raise ValueError("r must be >= 0")
    up = np.empty(a.size, a.dtype)
    lo = np.empty(a.size, a.dtype)
    if load().oracle_envelope(_code(a), _ptr(a), a.size, int(r), _ptr(up), _ptr(lo)) != 0:
        raise ValueError("oracle_envelope: bad arguments")
    return up, lo


def envelope_batched(packed, in_offsets, radii):
    """Envelope of each series of a packed buffer, packed the same way."""
    packed = np.ascontiguousarray(packed)
    up = np.empty_like(packed)
    lo = np.empty_like(packed)
    for k in range(len(radii)):
        s, e = int(in_offsets[k]), int(in_offsets[k + 1])
        up[s:e], lo[s:e] = envelope(packed[s:e], radii[k])
    return up, lo


def argnaive(a, w):
    """Leftmost locations of each window's max and min, from the definition
    (O(n*w))."""
    return _arg(load().oracle_argnaive, a, w)


def argdeque(a, w):
    """The same locations in linear time (monotonic deques of locations that
    keep equal values), pinned to :func:`argnaive`."""
    return _arg(load().oracle_argdeque, a, w)


class Stream:
    """The wedge kept across pushes: push(chunk) returns the windows that the
    chunk completes (zero stream latency, Section 1).

    export() gives the stream's state as (t, the last min(t, w-1) samples):
    every later window lies within the samples from t-w+1 on, so that is all
    a continuation needs.  Stream.resume(dtype, w, t, carry) rebuilds a wedge
    from it by pushing the carried samples, which complete no window (fewer
    than w of them), and counts samples from t."""

    def __init__(self, dtype, w):
        self.dtype = np.dtype(dtype)
        self.w = int(w)
        self._lib = load()
        self._h = self._lib.oracle_stream_create(DTYPES[self.dtype], self.w)
        if not self._h:
            raise ValueError("oracle_stream_create failed")
        self._t = 0
        self._carry = np.empty(0, self.dtype)

    @classmethod
    def resume(cls, dtype, w, t, carry):
        st = cls(dtype, w)
        carry = np.ascontiguousarray(carry, dtype=st.dtype)
        if carry.size != max(0, min(int(t), st.w - 1)):
            raise ValueError("carry must hold min(t, w-1) samples")
        mx, _ = st.push(carry)
        assert mx.size == 0
        st._t = int(t)
        return st

    def push(self, chunk):
        chunk = np.ascontiguousarray(chunk, dtype=self.dtype)
        cap = chunk.size
        mx = np.empty(cap, self.dtype)
        mn = np.empty(cap, self.dtype)
        k = self._lib.oracle_stream_push(self._h, _ptr(chunk), chunk.size, _ptr(mx), _ptr(mn))
        self._t += chunk.size
        keep = min(self._t, self.w - 1)
        self._carry = np.concatenate([self._carry, chunk])[len(self._carry) + chunk.size - keep:].copy()
        return mx[:k].copy(), mn[:k].copy()

    def export(self):
        return self._t, self._carry.copy()

    def stats(self):
        t, c, p = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        self._lib.oracle_stream_stats(self._h, ctypes.byref(t), ctypes.byref(c), ctypes.byref(p))
        return {"t": t.value, "comparisons": c.value, "peak": p.value}

    def close(self):
        if self._h:
            self._lib.oracle_stream_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _two_d(fn, a, wr, wc):
    a = np.ascontiguousarray(a)
    rows, cols = a.shape
    orr, occ = n_out(rows, wr), n_out(cols, wc)
    mx = np.empty((orr, occ), a.dtype)
    mn = np.empty((orr, occ), a.dtype)
    if orr and occ:
        if fn(_code(a), _ptr(a), rows, cols, cols, int(wr), int(wc), _ptr(mx), _ptr(mn), occ) != 0:
            raise ValueError("oracle 2-D: bad arguments")
    return mx, mn


def filter2d(a, wr, wc=None):
    """Rows first, then columns, each with the 1-D wedge filter."""
    return _two_d(load().oracle_filter2d, a, wr, wr if wc is None else wc)


def naive2d(a, wr, wc=None):
    """2-D definition: max/min over each wr x wc rectangle."""
    return _two_d(load().oracle_naive2d, a, wr, wr if wc is None else wc)


def morph2d(a, op, wr, wc=None, filt=None):
    """Grey-scale morphology with a wr x wc rectangle, valid windows:
    erosion = the min image of the 2-D filter, dilation = the max image,
    opening = dilation of the erosion, closing = erosion of the dilation.
    ``filt`` is the 2-D filter used (default :func:`filter2d`)."""
    wc = wr if wc is None else wc
    filt = filt or filter2d
    if op == "erode":
        return filt(a, wr, wc)[1]
    if op == "dilate":
        return filt(a, wr, wc)[0]
    first, second = (1, 0) if op == "open" else (0, 1)
    mid = filt(a, wr, wc)[first]
    if mid.size == 0:
        return np.empty((max(0, mid.shape[0] - wr + 1), max(0, mid.shape[1] - wc + 1)), a.dtype)
    return filt(mid, wr, wc)[second]


def out_offsets(in_offsets, windows):
    """Exclusive scan of max(0, n_k - w_k + 1): where each series' outputs go."""
    in_offsets = np.asarray(in_offsets, np.int64)
    windows = np.asarray(windows, np.int64)
    lens = np.diff(in_offsets)
    no = np.maximum(0, lens - windows + 1)
    out = np.zeros(len(windows) + 1, np.int64)
    np.cumsum(no, out=out[1:])
    return out


def batched(packed, in_offsets, windows, series=None):
    """Filter each series of a packed buffer independently.

    Returns ``(out_offsets, max, min)`` with the outputs packed the same way.
    ``series`` restricts the work to a subset of series indices (the other
    outputs are left as zeros).
    """
    packed = np.ascontiguousarray(packed)
    in_offsets = np.asarray(in_offsets, np.int64)
    windows = np.asarray(windows, np.int64)
    oo = out_offsets(in_offsets, windows)
    mx = np.zeros(int(oo[-1]), packed.dtype)
    mn = np.zeros(int(oo[-1]), packed.dtype)
    idx = range(len(windows)) if series is None else series
    for k in idx:
        a = packed[in_offsets[k]:in_offsets[k + 1]]
        M, N = wedge(a, windows[k])
        mx[oo[k]:oo[k + 1]] = M
        mn[oo[k]:oo[k + 1]] = N
    return oo, mx, mn
