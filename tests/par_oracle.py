"""Whole-array expected values at full size: the oracle called on
independent pieces in parallel threads (the ctypes calls release the GIL).

Each window's max and min depend only on its own w samples (Section 1
definition), so a piece of windows [s, e) is the oracle run on the inputs
[s, e + w - 1); pieces of a batch are whole series, pieces of an image are
bands of output rows with their w_rows - 1 halo rows.  Nothing here selects
a value itself: every expected value comes from an ``oracle`` function.
"""
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

import oracle

THREADS = max(1, min(16, os.cpu_count() or 1))


def _pool():
    return ThreadPoolExecutor(max_workers=THREADS)


def wedge(a, w, piece=1 << 23):
    """oracle.wedge(a, w) for the whole series, in pieces of windows."""
    a = np.ascontiguousarray(a)
    nout = oracle.n_out(a.size, w)
    mx = np.empty(nout, a.dtype)
    mn = np.empty(nout, a.dtype)

    def run(s):
        e = min(nout, s + piece)
        mx[s:e], mn[s:e] = oracle.wedge(a[s:e + w - 1], w)

    with _pool() as ex:
        list(ex.map(run, range(0, nout, piece)))
    return mx, mn


def batched(packed, in_offsets, windows):
    """oracle.batched over every series, series in parallel:
    ``(out_offsets, max, min)``."""
    packed = np.ascontiguousarray(packed)
    oo = oracle.out_offsets(in_offsets, windows)
    mx = np.zeros(int(oo[-1]), packed.dtype)
    mn = np.zeros(int(oo[-1]), packed.dtype)
    order = np.argsort(-np.diff(np.asarray(in_offsets)))  # longest first

    def run(k):
        if oo[k + 1] > oo[k]:
            mx[oo[k]:oo[k + 1]], mn[oo[k]:oo[k + 1]] = oracle.wedge(packed[in_offsets[k]:in_offsets[k + 1]],
                                                                    int(windows[k]))

    with _pool() as ex:
        list(ex.map(run, order))
    return oo, mx, mn


def filter2d(img, wr, wc=None, band=512):
    """oracle.filter2d(img, wr, wc) in bands of output rows."""
    wc = wr if wc is None else wc
    img = np.ascontiguousarray(img)
    orows, ocols = oracle.n_out(img.shape[0], wr), oracle.n_out(img.shape[1], wc)
    mx = np.empty((orows, ocols), img.dtype)
    mn = np.empty((orows, ocols), img.dtype)

    def run(r0):
        r1 = min(orows, r0 + band)
        mx[r0:r1], mn[r0:r1] = oracle.filter2d(img[r0:r1 + wr - 1], wr, wc)

    with _pool() as ex:
        list(ex.map(run, range(0, orows, band)))
    return mx, mn


def morph2d(img, op, wr, wc=None, band=512):
    """oracle.morph2d in bands of output rows (opening / closing need
    2 (w_rows - 1) halo rows)."""
    wc = wr if wc is None else wc
    img = np.ascontiguousarray(img)
    k = 1 if op in ("erode", "dilate") else 2
    orows = max(0, img.shape[0] - k * (wr - 1))
    ocols = max(0, img.shape[1] - k * (wc - 1))
    out = np.empty((orows, ocols), img.dtype)

    def run(r0):
        r1 = min(orows, r0 + band)
        out[r0:r1] = oracle.morph2d(img[r0:r1 + k * (wr - 1)], op, wr, wc)

    with _pool() as ex:
        list(ex.map(run, range(0, orows, band)))
    return out


def envelope_batched(packed, in_offsets, radii):
    """oracle.envelope over every series of a packed batch, in parallel."""
    packed = np.ascontiguousarray(packed)
    up = np.empty_like(packed)
    lo = np.empty_like(packed)

    def run(k):
        s, e = int(in_offsets[k]), int(in_offsets[k + 1])
        up[s:e], lo[s:e] = oracle.envelope(packed[s:e], int(radii[k]))

    with _pool() as ex:
        list(ex.map(run, range(len(radii))))
    return up, lo
