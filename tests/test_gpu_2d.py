"""GPU parity of the 2-D filter (rows, then columns) against the oracle."""
import numpy as np
import pytest

import oracle
from paper_cs_0610046_amd import binding as mm
from paper_cs_0610046_amd import synth
from gpu_util import assert_bits_equal, note, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(params=["fused", "unfused"])
def path2d(request, monkeypatch):
    """Both 2-D paths: the fused single pass (windows it fits) and rows then
    columns through intermediate images (MAXMIN_2D_FUSED=0)."""
    monkeypatch.setenv("MAXMIN_2D_FUSED", "1" if request.param == "fused" else "0")
    return request.param


def _image(rows, cols, dt, rng):
    if dt == np.uint16:
        return synth.uniform_u16((rows, cols), rng)
    if dt == np.int32:
        return rng.integers(-1000, 1000, (rows, cols)).astype(np.int32)
    return synth.gaussian_field(rows, cols, sigma=4.0, rng=rng).astype(dt)


@pytest.mark.parametrize("dt", [np.float32, np.float64, np.int32, np.uint16], ids=lambda d: np.dtype(d).name)
def test_2d_small_images(dt, path2d):
    rng = synth.rng_for("tests", 200)
    cases = [(1, 1, 1, 1), (5, 7, 2, 3), (64, 64, 3, 3), (100, 300, 15, 15), (257, 2100, 63, 63),
             (130, 3000, 7, 1500), (70, 50, 70, 1), (33, 4100, 1, 1025), (300, 40, 128 if dt != np.float64 else 64, 5),
             (700, 90, 200, 4), (20, 9000, 3, 3000), (9, 4200, 2, 4096), (6, 2049, 4, 2049), (150, 500, 40, 9),
             (200, 333, 49, 2), (7, 9000, 2, 6000), (5, 8200, 3, 8192)]
    for rows, cols, wr, wc in cases:
        if dt == np.uint16:
            a = synth.uniform_u16((rows, cols), rng)
        else:
            a = synth.gaussian_field(rows, cols, sigma=4.0, rng=rng).astype(dt) if dt != np.int32 else \
                rng.integers(-1000, 1000, (rows, cols)).astype(np.int32)
        note("2d dt=%s %dx%d w=%dx%d" % (np.dtype(dt).name, rows, cols, wr, wc))
        x = to_dev(a)
        gmx, gmn = mm.maxmin_filter_2d(x, wr, wc)
        omx, omn = oracle.filter2d(a, wr, wc)
        assert_bits_equal(to_host(gmx, dt), omx, "2d max")
        assert_bits_equal(to_host(gmn, dt), omn, "2d min")
        if wr in (3, 15, 63):  # one output only (each path's null-image handling)
            ox, _ = mm.maxmin_filter_2d(x, wr, wc, which="max")
            _, on = mm.maxmin_filter_2d(x, wr, wc, which="min")
            assert_bits_equal(to_host(ox, dt), omx, "2d max-only")
            assert_bits_equal(to_host(on, dt), omn, "2d min-only")


def test_2d_strided_input(path2d):
    import torch
    rng = synth.rng_for("tests", 201)
    a = synth.gaussian_field(200, 300, sigma=5.0, rng=rng)
    big = to_dev(np.pad(a, ((0, 0), (0, 37))))
    view = big[:, :300]
    note("2d strided 200x300 ld=337")
    gmx, gmn = mm.maxmin_filter_2d(view, 15, 9)
    torch.cuda.synchronize()
    omx, omn = oracle.filter2d(a, 15, 9)
    assert_bits_equal(to_host(gmx, np.float32), omx, "strided max")
    assert_bits_equal(to_host(gmn, np.float32), omn, "strided min")


@pytest.mark.parametrize("dt", [np.float32, np.float64, np.int32, np.uint16], ids=lambda d: np.dtype(d).name)
def test_2d_fused_edges(dt, monkeypatch):
    """The fused pass at its limits: every column-block size (w_rows 1..64)
    with the widest row window it takes (64 V + 1) and narrow ones, strips
    and bands with ragged ends, bands of 1..9 rows (every band re-reads its
    w_rows-1 halo rows), unaligned row pitch and outputs (scalar path), a
    single output pixel, and max-only / min-only."""
    import torch
    rng = synth.rng_for("tests", 202)
    monkeypatch.setenv("MAXMIN_2D_FUSED", "1")  # also where the planner prefers rows-then-columns
    widest = {1: 257, 2: 257, 3: 257, 4: 257, 5: 257, 7: 257, 8: 129, 15: 129, 16: 65, 31: 65, 32: 65,
              63: 65, 64: 65}
    for wr, wcmax in widest.items():
        for wc in sorted({1, 2, 3, wcmax}):
            assert mm.maxmin_plan_2d(dt, wr, wc) == mm.PLAN_2D_FUSED
            rows = wr + int(rng.integers(0, 40))
            cols = wc + int(rng.integers(0, 700))
            a = _image(rows, cols, dt, rng)
            for band in (None, "1", "7"):
                if band is None:
                    monkeypatch.delenv("MAXMIN_2D_BAND", raising=False)
                else:
                    monkeypatch.setenv("MAXMIN_2D_BAND", band)
                note("2d fused dt=%s %dx%d w=%dx%d band=%s" % (np.dtype(dt).name, rows, cols, wr, wc, band))
                gmx, gmn = mm.maxmin_filter_2d(to_dev(a), wr, wc)
                omx, omn = oracle.filter2d(a, wr, wc)
                assert_bits_equal(to_host(gmx, dt), omx, "fused max %dx%d" % (wr, wc))
                assert_bits_equal(to_host(gmn, dt), omn, "fused min %dx%d" % (wr, wc))
    monkeypatch.delenv("MAXMIN_2D_BAND", raising=False)
    assert mm.maxmin_plan_2d(dt, 65, 3) == mm.PLAN_2D_ROWS_COLS
    assert mm.maxmin_plan_2d(dt, 63, 66) == mm.PLAN_2D_ROWS_COLS
    # unaligned pitch, offset outputs, one output only, a single pixel
    a = _image(70, 1001, dt, rng)
    big = to_dev(np.pad(a, ((0, 0), (0, 3))))
    view = big[:, :1001]
    for wr, wc in ((3, 3), (15, 15), (63, 63)):
        orow, ocol = 70 - wr + 1, 1001 - wc + 1
        tdt = view.dtype
        bx = torch.zeros((orow, ocol + 5), dtype=tdt, device="cuda")
        bn = torch.zeros((orow, ocol + 5), dtype=tdt, device="cuda")
        note("2d fused unaligned dt=%s w=%dx%d" % (np.dtype(dt).name, wr, wc))
        mm.maxmin_filter_2d(view, wr, wc, bx[:, 1:ocol + 1], bn[:, 3:ocol + 3])
        gx, none = mm.maxmin_filter_2d(view, wr, wc, which="max")
        none2, gn = mm.maxmin_filter_2d(view, wr, wc, which="min")
        torch.cuda.synchronize()
        assert none is None and none2 is None
        omx, omn = oracle.filter2d(a, wr, wc)
        assert_bits_equal(to_host(bx[:, 1:ocol + 1], dt), omx, "unaligned max")
        assert_bits_equal(to_host(bn[:, 3:ocol + 3], dt), omn, "unaligned min")
        assert_bits_equal(to_host(gx, dt), omx, "max-only")
        assert_bits_equal(to_host(gn, dt), omn, "min-only")
    a = _image(5, 9, dt, rng)
    gmx, gmn = mm.maxmin_filter_2d(to_dev(a), 5, 9)
    omx, omn = oracle.filter2d(a, 5, 9)
    assert_bits_equal(to_host(gmx, dt), omx, "single pixel max")
    assert_bits_equal(to_host(gmn, dt), omn, "single pixel min")


@pytest.mark.parametrize("cpass", ["block", "stream", "ring", "ring-v1d8", "ring-v1d16", "ring-v2d8", "ring-v2d16",
                                   "ring-v4d8"])
@pytest.mark.parametrize("dt", [np.float32, np.float64, np.int32, np.uint16], ids=lambda d: np.dtype(d).name)
def test_2d_column_passes(dt, cpass, monkeypatch):
    """Rows then columns with each column pass forced (blocks of w_rows rows,
    the fused kernel's streaming column filter, the streaming LDS ring with
    its default and every instantiated lane width V and prefetch depth D):
    every window size class up to 64 rows, odd and even output widths (lane
    groups cut by the image edge), bands of one and of several blocks (every
    band re-reads w_rows - 1 rows), offset outputs (stores that cannot be
    widened) and one-output calls."""
    import torch
    rng = synth.rng_for("tests", 203)
    monkeypatch.setenv("MAXMIN_2D_FUSED", "0")
    monkeypatch.setenv("MAXMIN_COLS_PASS", cpass.split("-")[0])
    if "-" in cpass:
        v, d = cpass.split("-")[1][1:].split("d")
        monkeypatch.setenv("MAXMIN_COLS_V", v)
        monkeypatch.setenv("MAXMIN_COLS_D", d)
    for wr in (1, 2, 15, 16, 17, 31, 33, 48, 49, 63, 64):
        wc = int(rng.integers(1, 9))
        rows = wr + int(rng.integers(0, 300))
        cols = wc + int(rng.integers(0, 400))
        a = _image(rows, cols, dt, rng)
        for band in (None, "1", str(3 * wr)):
            if band is None:
                monkeypatch.delenv("MAXMIN_COLS_BAND", raising=False)
            else:
                monkeypatch.setenv("MAXMIN_COLS_BAND", band)
            note("2d cols=%s dt=%s %dx%d w=%dx%d band=%s" % (cpass, np.dtype(dt).name, rows, cols, wr, wc, band))
            gmx, gmn = mm.maxmin_filter_2d(to_dev(a), wr, wc)
            omx, omn = oracle.filter2d(a, wr, wc)
            assert_bits_equal(to_host(gmx, dt), omx, "cols %s max %dx%d" % (cpass, wr, wc))
            assert_bits_equal(to_host(gmn, dt), omn, "cols %s min %dx%d" % (cpass, wr, wc))
        monkeypatch.delenv("MAXMIN_COLS_BAND", raising=False)
        orow, ocol = rows - wr + 1, cols - wc + 1
        x = to_dev(a)
        bx = torch.zeros((orow, ocol + 5), dtype=x.dtype, device="cuda")
        bn = torch.zeros((orow, ocol + 5), dtype=x.dtype, device="cuda")
        note("2d cols=%s dt=%s offset outputs w=%d" % (cpass, np.dtype(dt).name, wr))
        mm.maxmin_filter_2d(x, wr, wc, bx[:, 1:ocol + 1], bn[:, 3:ocol + 3])
        gx, _ = mm.maxmin_filter_2d(x, wr, wc, which="max")
        _, gn = mm.maxmin_filter_2d(x, wr, wc, which="min")
        torch.cuda.synchronize()
        omx, omn = oracle.filter2d(a, wr, wc)
        assert_bits_equal(to_host(bx[:, 1:ocol + 1], dt), omx, "offset max")
        assert_bits_equal(to_host(bn[:, 3:ocol + 3], dt), omn, "offset min")
        assert_bits_equal(to_host(gx, dt), omx, "max-only")
        assert_bits_equal(to_host(gn, dt), omn, "min-only")
    # a single output column (every lane group cut by the image edge) and
    # one or two output rows
    for wr in (16, 33, 64):
        for rows, cols, wc in ((wr, 2, 2), (wr + 1, 3, 3), (wr + 1, 1, 1)):
            a = _image(rows, cols, dt, rng)
            note("2d cols=%s dt=%s tiny %dx%d w=%dx%d" % (cpass, np.dtype(dt).name, rows, cols, wr, wc))
            gmx, gmn = mm.maxmin_filter_2d(to_dev(a), wr, wc)
            omx, omn = oracle.filter2d(a, wr, wc)
            assert_bits_equal(to_host(gmx, dt), omx, "tiny max %dx%d" % (wr, wc))
            assert_bits_equal(to_host(gmn, dt), omn, "tiny min %dx%d" % (wr, wc))
