"""GPU parity of the centered envelopes (windows [i-r, i+r] truncated at the
series ends) against the oracle's definition, bit-exact: every dtype,
radii around the tile / chunk boundaries and the end-scan tile, series
shorter than the window, misaligned buffers, and the batched call."""
import numpy as np
import pytest

import oracle
from paper_cs_0610046_amd import binding as mm
from paper_cs_0610046_amd import synth
from gpu_util import assert_bits_equal, note, to_dev, to_host

pytestmark = pytest.mark.gpu

DTS = [np.float32, np.float64, np.int32, np.uint16]


def _gen(n, dt, rng):
    if dt in (np.float32, np.float64):
        return synth.random_walk(n, dt, rng)
    return synth.small_alphabet(n, 3000, dt, rng)


def _expected(a, r):
    n = a.size
    if n * (2 * r + 1) <= 4e8:
        return oracle.envelope(a, r)
    # large cases: the valid-window wedge inside, running max/min at the ends
    up, lo = np.empty_like(a), np.empty_like(a)
    mx, mn = oracle.wedge(a, 2 * r + 1)
    up[r:n - r], lo[r:n - r] = mx, mn
    pm, pn = np.maximum.accumulate(a), np.minimum.accumulate(a)
    sm, sn = np.maximum.accumulate(a[::-1])[::-1], np.minimum.accumulate(a[::-1])[::-1]
    i = np.arange(n)
    left, right = i < r, i > n - 1 - r
    up[left], lo[left] = pm[np.minimum(i[left] + r, n - 1)], pn[np.minimum(i[left] + r, n - 1)]
    both = left & right
    up[right & ~left], lo[right & ~left] = sm[i[right & ~left] - r], sn[i[right & ~left] - r]
    up[both], lo[both] = a.max(), a.min()
    return up, lo


@pytest.mark.parametrize("dt", DTS, ids=lambda d: np.dtype(d).name)
def test_envelope_single(dt):
    import torch
    rng = synth.rng_for("tests", 700)
    for r in (0, 1, 2, 5, 100, 511, 512, 513, 1024, 2047, 2048, 5000, 40000):
        for n in sorted({1, 2, 2 * r, 2 * r + 1, 2 * r + 2, 5000, 100003}):
            if n < 1:
                continue
            a = _gen(n, dt, rng)
            note("envelope dt=%s n=%d r=%d" % (np.dtype(dt).name, n, r))
            up, lo = mm.maxmin_envelope(to_dev(a), r)
            torch.cuda.synchronize()
            mm.maxmin_check_stream()
            eu, el = _expected(a, r)
            assert_bits_equal(to_host(up, dt), eu, "upper n=%d r=%d" % (n, r))
            assert_bits_equal(to_host(lo, dt), el, "lower n=%d r=%d" % (n, r))


def test_envelope_misaligned_and_huge_radius():
    import torch
    rng = synth.rng_for("tests", 701)
    for dt in DTS:
        a = _gen(30001, dt, rng)
        for off in (1, 3):
            for r in (7, 700):
                buf = to_dev(np.concatenate([np.zeros(off, dt), a]))
                ob = torch.empty(a.size + 8, dtype=buf.dtype, device="cuda")
                ol = torch.empty(a.size + 8, dtype=buf.dtype, device="cuda")
                note("envelope misaligned dt=%s off=%d r=%d" % (np.dtype(dt).name, off, r))
                mm.maxmin_envelope(buf[off:], r, ob[off + 1:off + 1 + a.size], ol[2:2 + a.size])
                torch.cuda.synchronize()
                eu, el = oracle.envelope(a, r)
                assert_bits_equal(to_host(ob[off + 1:off + 1 + a.size], dt), eu, "upper")
                assert_bits_equal(to_host(ol[2:2 + a.size], dt), el, "lower")
        up, lo = mm.maxmin_envelope(to_dev(a[:999]), 1 << 62)
        torch.cuda.synchronize()
        assert np.all(to_host(up, dt) == a[:999].max()) and np.all(to_host(lo, dt) == a[:999].min())


def test_envelope_batched():
    import torch
    rng = synth.rng_for("tests", 702)
    S = 500
    lens = rng.integers(0, 5000, S)
    radii = rng.integers(0, 300, S).astype(np.int64)
    radii[::7] = lens[::7] + 5  # radius beyond the series
    offs = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    for dt in (np.float32, np.uint16):
        packed = _gen(int(offs[-1]), dt, rng)
        d_off, d_r = torch.from_numpy(offs).cuda(), torch.from_numpy(radii).cuda()
        x = to_dev(packed)
        note("envelope batched dt=%s" % np.dtype(dt).name)
        eu, el = oracle.envelope_batched(packed, offs, radii)
        for rep in range(2):  # the second call replays the captured batched filter
            up, lo = mm.maxmin_envelope_batched(x, d_off, d_r)
            torch.cuda.synchronize()
            mm.maxmin_check_stream()
            assert_bits_equal(to_host(up, dt), eu, "batched upper rep %d" % rep)
            assert_bits_equal(to_host(lo, dt), el, "batched lower rep %d" % rep)


@pytest.mark.parametrize("dt", [np.float32, np.float64, np.int32, np.uint16], ids=lambda d: np.dtype(d).name)
def test_envelope_batched_short_and_long(dt):
    """Series served whole by one wavefront (n <= 16384, r <= 256) mixed with
    series that take the batched filter plus end scans (longer, or wider
    radius): lengths at the 512-output segment edges and the short limit,
    radius 0, radius at the limit, radius past the series, single samples,
    empty series."""
    import torch
    rng = synth.rng_for("tests", 703)
    lens = [1, 2, 511, 512, 513, 1024, 1500, 16384, 16385, 20000, 0, 3, 777, 4096, 16384, 9000, 300, 1]
    radii = [0, 0, 3, 256, 255, 100, 257, 256, 10, 256, 5, 2, 777, 1000, 0, 300, 150, 400]
    lens += list(rng.integers(1, 3000, 40))
    radii += list(rng.integers(0, 400, 40))
    lens, radii = np.array(lens, np.int64), np.array(radii, np.int64)
    offs = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    packed = _gen(int(offs[-1]), dt, rng)
    d_off, d_r = torch.from_numpy(offs).cuda(), torch.from_numpy(radii).cuda()
    x = to_dev(packed)
    note("envelope batched short/long dt=%s" % np.dtype(dt).name)
    eu, el = oracle.envelope_batched(packed, offs, radii)
    up, lo = mm.maxmin_envelope_batched(x, d_off, d_r)
    torch.cuda.synchronize()
    mm.maxmin_check_stream()
    assert_bits_equal(to_host(up, dt), eu, "short/long upper")
    assert_bits_equal(to_host(lo, dt), el, "short/long lower")
