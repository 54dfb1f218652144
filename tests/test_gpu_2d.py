"""GPU parity of the 2-D filter (rows, then columns) against the oracle."""
import numpy as np
import pytest

import oracle
from paper_cs_0610046_amd import binding as mm
from paper_cs_0610046_amd import synth
from gpu_util import assert_bits_equal, note, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dt", [np.float32, np.float64, np.int32, np.uint16], ids=lambda d: np.dtype(d).name)
def test_2d_small_images(dt):
    rng = synth.rng_for("tests", 200)
    cases = [(1, 1, 1, 1), (5, 7, 2, 3), (64, 64, 3, 3), (100, 300, 15, 15), (257, 2100, 63, 63),
             (130, 3000, 7, 1500), (70, 50, 70, 1), (33, 4100, 1, 1025), (300, 40, 128 if dt != np.float64 else 64, 5),
             (700, 90, 200, 4), (20, 9000, 3, 3000), (9, 4200, 2, 4096), (6, 2049, 4, 2049)]
    for rows, cols, wr, wc in cases:
        if dt == np.uint16:
            a = synth.uniform_u16((rows, cols), rng)
        else:
            a = synth.gaussian_field(rows, cols, sigma=4.0, rng=rng).astype(dt) if dt != np.int32 else \
                rng.integers(-1000, 1000, (rows, cols)).astype(np.int32)
        note("2d dt=%s %dx%d w=%dx%d" % (np.dtype(dt).name, rows, cols, wr, wc))
        gmx, gmn = mm.maxmin_filter_2d(to_dev(a), wr, wc)
        omx, omn = oracle.filter2d(a, wr, wc)
        assert_bits_equal(to_host(gmx, dt), omx, "2d max")
        assert_bits_equal(to_host(gmn, dt), omn, "2d min")


def test_2d_strided_input():
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
