"""Parity at the benchmark's full sizes, in the launch configuration the
benchmark times: outputs are sampled (the oracle's definition computes each
sampled window on its own) plus properties that hold at any size."""
import numpy as np
import pytest

import oracle
from paper_cs_0610046_amd import binding as mm
from paper_cs_0610046_amd import synth
from gpu_util import assert_bits_equal, note, to_dev, to_host

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(900)]


def sample_check(a, w, gmx, gmn, rng, k=4000, what=""):
    nout = a.size - w + 1
    idx = np.unique(np.concatenate([rng.integers(0, nout, k), [0, 1, nout - 2, nout - 1],
                                    np.arange(0, nout, max(1, nout // 64))]))
    idx = idx[(idx >= 0) & (idx < nout)]
    emx = np.empty(idx.size, a.dtype)
    emn = np.empty(idx.size, a.dtype)
    for i, j in enumerate(idx):
        M, N = oracle.naive(a[j:j + w], w)
        emx[i], emn[i] = M[0], N[0]
    assert_bits_equal(gmx[idx], emx, what + " sampled max")
    assert_bits_equal(gmn[idx], emn, what + " sampled min")


def window_properties(a, w, gmx, gmn, what=""):
    """max/min are non-negative/non-positive distance from every window's end
    points, and consecutive windows differ only through the samples that
    enter or leave (the running max changes only if one of them is involved)."""
    nout = a.size - w + 1
    assert gmx.size == nout and gmn.size == nout
    assert np.all(gmx >= a[:nout]) and np.all(gmx >= a[w - 1:]), what
    assert np.all(gmn <= a[:nout]) and np.all(gmn <= a[w - 1:]), what
    assert np.all(gmx >= gmn)
    d = gmx[1:] != gmx[:-1]
    # if the max changed, either the entering sample is the new max or the
    # leaving sample was the old max
    ent, lea = a[w:], a[:nout - 1]
    assert np.all(~d | (gmx[1:] == ent) | (gmx[:-1] == lea)), what


@pytest.mark.parametrize("kind", ["walk", "pwm", "ramp"])
def test_large_series_f32(kind):
    import torch
    rng = synth.rng_for("tests", 300)
    note("full-size generate kind=%s n=2^28" % kind)
    a = synth.large_series(kind)
    x = to_dev(a)
    for w in (16, 256, 4096, 65536):
        note("full-size f32 kind=%s w=%d" % (kind, w))
        mx, mn = mm.maxmin_filter(x, w)
        torch.cuda.synchronize()
        mm.maxmin_check_stream()
        gmx, gmn = to_host(mx, np.float32), to_host(mn, np.float32)
        sample_check(a, w, gmx, gmn, rng, what="%s w=%d" % (kind, w))
        window_properties(a, w, gmx, gmn, what="%s w=%d" % (kind, w))
        if kind == "ramp":
            assert_bits_equal(gmx, a[w - 1:], "ramp max closed form")
            assert_bits_equal(gmn, a[:a.size - w + 1], "ramp min closed form")
        del mx, mn


def test_large_series_f64_i32():
    import torch
    rng = synth.rng_for("tests", 301)
    note("full-size generate f64 walk")
    a = synth.random_walk(1 << 28, np.float64, synth.rng_for("large", 0))
    for arr in (a, synth.large_series("i32")):
        x = to_dev(arr)
        for w in (16, 65536):
            note("full-size %s w=%d" % (arr.dtype, w))
            mx, mn = mm.maxmin_filter(x, w)
            torch.cuda.synchronize()
            gmx, gmn = to_host(mx, arr.dtype), to_host(mn, arr.dtype)
            sample_check(arr, w, gmx, gmn, rng, k=1500, what="%s w=%d" % (arr.dtype, w))
            del mx, mn
        del x


def test_plain_config_full():
    """n = 2^20 float32 uniform, w = 64: the oracle finishes it whole."""
    import torch
    a = synth.uniform01(1 << 20)
    note("plain n=2^20 w=64")
    mx, mn = mm.maxmin_filter(to_dev(a), 64)
    torch.cuda.synchronize()
    omx, omn = oracle.wedge(a, 64)
    assert_bits_equal(to_host(mx, np.float32), omx, "plain max")
    assert_bits_equal(to_host(mn, np.float32), omn, "plain min")
