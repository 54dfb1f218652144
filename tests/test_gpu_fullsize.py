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


def test_batched_config_full():
    """The benchmark's batch (10,000 float32 walks, lengths log-uniform in
    [1e3, 1e6], windows in [2, 1024]) in one batched call: 24 whole series
    (the shortest, the longest and random ones) against the oracle, and
    every series' first and last window against the definition."""
    import torch
    rng = np.random.default_rng(11)
    note("full-size batched generate")
    packed, offs, wins = synth.batched_series()
    oo = mm.maxmin_out_offsets(offs, wins)
    x = torch.from_numpy(packed).cuda()
    d_off, d_w, d_oo = (torch.from_numpy(v).cuda() for v in (offs, wins, oo))
    note("full-size batched run S=%d elements=%d" % (wins.size, packed.size))
    gmx, gmn = mm.maxmin_filter_batched(x, d_off, d_w, d_oo)
    torch.cuda.synchronize()
    mm.maxmin_check_stream()
    gmx, gmn = gmx.cpu().numpy(), gmn.cpu().numpy()
    lens = np.diff(offs)
    pick = np.unique(np.concatenate([[np.argmin(lens), np.argmax(lens)], rng.integers(0, wins.size, 22)]))
    for k in pick:
        a = packed[offs[k]:offs[k + 1]]
        omx, omn = oracle.wedge(a, int(wins[k]))
        assert_bits_equal(gmx[oo[k]:oo[k + 1]], omx, "series %d max" % k)
        assert_bits_equal(gmn[oo[k]:oo[k + 1]], omn, "series %d min" % k)
    for k in range(wins.size):
        a, w = packed[offs[k]:offs[k + 1]], int(wins[k])
        if oo[k + 1] == oo[k]:
            continue
        for j, o in ((0, oo[k]), (a.size - w, oo[k + 1] - 1)):
            assert gmx[o] == a[j:j + w].max() and gmn[o] == a[j:j + w].min(), (k, j)


@pytest.mark.parametrize("dt", [np.float32, np.uint16], ids=["f32", "u16"])
def test_image_config_full(dt, monkeypatch):
    """8192 x 8192 (float32 Gaussian field; uint16 uniform), w x w windows
    3 / 15 / 63 as the benchmark runs them: 3000 sampled output pixels
    against the definition (max/min over the w x w input block), and the
    fused pass and rows-then-columns agree bit for bit on the whole image."""
    import torch
    rng = np.random.default_rng(12)
    note("full-size image generate %s" % np.dtype(dt).name)
    img = synth.gaussian_field(8192, 8192) if dt == np.float32 else synth.uniform_u16((8192, 8192))
    x = to_dev(img)
    for w in (3, 15, 63):
        note("full-size image %s w=%d" % (np.dtype(dt).name, w))
        gmx, gmn = mm.maxmin_filter_2d(x, w, w)
        torch.cuda.synchronize()
        hx, hn = to_host(gmx, dt), to_host(gmn, dt)
        o = 8192 - w + 1
        ii, jj = rng.integers(0, o, 3000), rng.integers(0, o, 3000)
        ii[:4], jj[:4] = [0, 0, o - 1, o - 1], [0, o - 1, 0, o - 1]
        for i, j in zip(ii, jj):
            blk = img[i:i + w, j:j + w]
            assert hx[i, j] == blk.max() and hn[i, j] == blk.min(), (w, i, j)
        # the path the planner did not take (both serve these windows)
        monkeypatch.setenv("MAXMIN_2D_FUSED", "0" if mm.maxmin_plan_2d(dt, w, w) == mm.PLAN_2D_FUSED else "1")
        ax, an = mm.maxmin_filter_2d(x, w, w)
        torch.cuda.synchronize()
        monkeypatch.delenv("MAXMIN_2D_FUSED")
        assert torch.equal(ax, gmx) and torch.equal(an, gmn), "paths differ at w=%d" % w
        del gmx, gmn, ax, an


def test_envelope_config_full():
    """100,000 float32 walks of 1024 samples, radius uniform in [10, 100],
    one batched call as the benchmark runs it: 300 whole series against the
    oracle's envelope."""
    import torch
    rng = np.random.default_rng(13)
    S, L = 100000, 1024
    radii = rng.integers(10, 101, S).astype(np.int64)
    offs = np.arange(S + 1, dtype=np.int64) * L
    packed = synth.random_walk(S * L, np.float32, synth.rng_for("envelope", 0))
    x = to_dev(packed)
    d_off, d_r = torch.from_numpy(offs).cuda(), torch.from_numpy(radii).cuda()
    note("full-size envelope S=%d" % S)
    up, lo = mm.maxmin_envelope_batched(x, d_off, d_r)
    torch.cuda.synchronize()
    up, lo = up.cpu().numpy(), lo.cpu().numpy()
    for k in np.unique(np.concatenate([[0, S - 1], rng.integers(0, S, 298)])):
        a = packed[offs[k]:offs[k + 1]]
        eu, el = oracle.envelope(a, int(radii[k]))
        assert_bits_equal(up[offs[k]:offs[k + 1]], eu, "series %d upper" % k)
        assert_bits_equal(lo[offs[k]:offs[k + 1]], el, "series %d lower" % k)


def test_morphology_config_full():
    """Opening of the 8192 x 8192 float32 field with a 15 x 15 square (the
    benchmark's morphology call): 300 sampled output pixels against the
    definition on their 29 x 29 input patch (dilation of the erosion)."""
    import torch
    from numpy.lib.stride_tricks import sliding_window_view
    rng = np.random.default_rng(14)
    img = synth.gaussian_field(8192, 8192)
    x = to_dev(img)
    note("full-size morphology opening 15x15")
    out = mm.maxmin_morph_2d(x, "open", 15, 15)
    torch.cuda.synchronize()
    h = to_host(out, np.float32)
    o = 8192 - 2 * 14
    assert h.shape == (o, o)
    for i, j in zip(rng.integers(0, o, 300), rng.integers(0, o, 300)):
        patch = img[i:i + 29, j:j + 29]
        ero = sliding_window_view(patch, (15, 15)).min(axis=(2, 3))
        assert h[i, j] == ero.max(), (i, j)
