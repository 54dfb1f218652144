"""Helpers for the GPU parity tests (bit-exact comparison with the oracle)."""
import sys

import numpy as np

_UINT = {1: np.uint8, 2: np.uint16, 4: np.uint32, 8: np.uint64}


def note(msg):
    """Name the case about to run on the GPU (flushed, so a crash still shows it)."""
    print("[gpu case] " + msg, flush=True)
    sys.stdout.flush()


def to_dev(a):
    import torch
    if a.dtype == np.uint16:
        return torch.from_numpy(a.view(np.int16).copy()).view(torch.uint16).cuda()
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def to_host(t, dtype):
    import torch
    t = t.detach().cpu()
    if t.dtype == torch.uint16:
        return t.view(torch.int16).numpy().view(np.uint16)
    return t.numpy().astype(dtype, copy=False)


def bits(a):
    a = np.ascontiguousarray(a)
    return a.view(_UINT[a.dtype.itemsize])


def assert_bits_equal(got, exp, what=""):
    got = np.asarray(got)
    exp = np.asarray(exp)
    assert got.shape == exp.shape, "%s: shape %s vs %s" % (what, got.shape, exp.shape)
    if got.size == 0:
        return
    gb, eb = bits(got), bits(exp)
    bad = np.nonzero(gb.ravel() != eb.ravel())[0]
    assert bad.size == 0, "%s: %d mismatches, first at %d: got %r expected %r" % (
        what, bad.size, bad[0], got.ravel()[bad[0]], exp.ravel()[bad[0]])
