"""Parity at the benchmark's full sizes, in the launch configuration the
benchmark times: every output element against the oracle (run on pieces in
parallel threads, ``par_oracle``), plus closed forms where the input has
them."""
import numpy as np
import pytest

import par_oracle
from paper_cs_0610046_amd import binding as mm
from paper_cs_0610046_amd import synth
from gpu_util import assert_bits_equal, note, to_dev, to_host

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(900)]

WINDOWS = (16, 256, 4096, 65536)


def _whole(x, a, what):
    """Filter the device series x (host copy a) at every benchmark window and
    compare both outputs with the oracle element by element."""
    import torch
    for w in WINDOWS:
        note("full-size %s w=%d" % (what, w))
        mx, mn = mm.maxmin_filter(x, w)
        torch.cuda.synchronize()
        mm.maxmin_check_stream()
        gmx, gmn = to_host(mx, a.dtype), to_host(mn, a.dtype)
        del mx, mn
        emx, emn = par_oracle.wedge(a, w)
        assert_bits_equal(gmx, emx, "%s w=%d max" % (what, w))
        assert_bits_equal(gmn, emn, "%s w=%d min" % (what, w))
        yield w, gmx, gmn


@pytest.mark.parametrize("kind", ["walk", "pwm", "ramp"])
def test_large_series_f32(kind):
    """n = 2^28 float32: random walk, piecewise monotone, strictly
    increasing ramp; windows 16, 256, 4096, 65536."""
    note("full-size generate kind=%s n=2^28" % kind)
    a = synth.large_series(kind)
    x = to_dev(a)
    for w, gmx, gmn in _whole(x, a, "f32 " + kind):
        if kind == "ramp":  # closed form: the window's last and first sample
            assert_bits_equal(gmx, a[w - 1:], "ramp max closed form")
            assert_bits_equal(gmn, a[:a.size - w + 1], "ramp min closed form")


@pytest.mark.parametrize("dt", ["f64", "i32"])
def test_large_series_f64_i32(dt):
    """The float64 copy of the walk and the int32 uniform series, n = 2^28
    (2 GiB of float64: byte offsets past 2^31), all four windows."""
    note("full-size generate %s n=2^28" % dt)
    a = synth.random_walk(1 << 28, np.float64, synth.rng_for("large", 0)) if dt == "f64" \
        else synth.large_series("i32")
    x = to_dev(a)
    for _ in _whole(x, a, dt):
        pass


def test_plain_config_full():
    """n = 2^20 float32 uniform, w = 64."""
    import torch
    a = synth.uniform01(1 << 20)
    note("plain n=2^20 w=64")
    mx, mn = mm.maxmin_filter(to_dev(a), 64)
    torch.cuda.synchronize()
    omx, omn = par_oracle.wedge(a, 64)
    assert_bits_equal(to_host(mx, np.float32), omx, "plain max")
    assert_bits_equal(to_host(mn, np.float32), omn, "plain min")


def test_batched_config_full():
    """The benchmark's batch (10,000 float32 walks, lengths log-uniform in
    [1e3, 1e6], windows in [2, 1024]) in one batched call, as the benchmark
    replays it: every series against the oracle."""
    import torch
    note("full-size batched generate")
    packed, offs, wins = synth.batched_series()
    oo = mm.maxmin_out_offsets(offs, wins)
    x = torch.from_numpy(packed).cuda()
    d_off, d_w, d_oo = (torch.from_numpy(v).cuda() for v in (offs, wins, oo))
    total = int(oo[-1])
    gmx = torch.empty(total, device="cuda")
    gmn = torch.empty(total, device="cuda")
    for rep in range(2):  # first call captures the graph, the second replays it
        note("full-size batched run %d S=%d elements=%d" % (rep, wins.size, packed.size))
        gmx.fill_(0)
        gmn.fill_(0)
        mm.maxmin_filter_batched(x, d_off, d_w, d_oo, gmx, gmn)
        torch.cuda.synchronize()
        mm.maxmin_check_stream()
        hx, hn = gmx.cpu().numpy(), gmn.cpu().numpy()
        if rep == 0:
            eoo, emx, emn = par_oracle.batched(packed, offs, wins)
            assert np.array_equal(eoo, oo)
        assert_bits_equal(hx, emx, "batched max (call %d)" % rep)
        assert_bits_equal(hn, emn, "batched min (call %d)" % rep)


@pytest.mark.parametrize("dt", [np.float32, np.uint16], ids=["f32", "u16"])
def test_image_config_full(dt, monkeypatch):
    """8192 x 8192 (float32 Gaussian field; uint16 uniform), w x w windows
    3 / 15 / 63: the whole output of the planned path and of the other path
    against the oracle."""
    import torch
    note("full-size image generate %s" % np.dtype(dt).name)
    img = synth.gaussian_field(8192, 8192) if dt == np.float32 else synth.uniform_u16((8192, 8192))
    x = to_dev(img)
    for w in (3, 15, 63):
        emx, emn = par_oracle.filter2d(img, w)
        planned = mm.maxmin_plan_2d(dt, w, w)
        for force in (None, "0" if planned == mm.PLAN_2D_FUSED else "1"):
            if force is None:
                monkeypatch.delenv("MAXMIN_2D_FUSED", raising=False)
            else:
                monkeypatch.setenv("MAXMIN_2D_FUSED", force)
            note("full-size image %s w=%d force=%s" % (np.dtype(dt).name, w, force))
            gmx, gmn = mm.maxmin_filter_2d(x, w, w)
            torch.cuda.synchronize()
            assert_bits_equal(to_host(gmx, dt), emx, "image w=%d force=%s max" % (w, force))
            assert_bits_equal(to_host(gmn, dt), emn, "image w=%d force=%s min" % (w, force))
            del gmx, gmn


def test_envelope_config_full():
    """100,000 float32 walks of 1024 samples, radius uniform in [10, 100],
    one batched call as the benchmark runs it: every series against the
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
    eu, el = par_oracle.envelope_batched(packed, offs, radii)
    assert_bits_equal(to_host(up, np.float32), eu, "envelope upper")
    assert_bits_equal(to_host(lo, np.float32), el, "envelope lower")


def test_morphology_config_full():
    """Opening of the 8192 x 8192 float32 field with a 15 x 15 square (the
    benchmark's morphology call): the whole output against the oracle."""
    import torch
    img = synth.gaussian_field(8192, 8192)
    x = to_dev(img)
    note("full-size morphology opening 15x15")
    out = mm.maxmin_morph_2d(x, "open", 15, 15)
    torch.cuda.synchronize()
    assert_bits_equal(to_host(out, np.float32), par_oracle.morph2d(img, "open", 15), "opening 15x15")
