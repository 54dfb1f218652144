"""The full-size tests' parallel oracle (pieces of windows, whole series,
bands of rows) returns exactly what the oracle returns in one call."""
import numpy as np

import oracle
import par_oracle
from paper_cs_0610046_amd import synth


def test_pieces_equal_one_call():
    rng = synth.rng_for("tests", 910)
    a = synth.random_walk(300001, np.float32, rng)
    for w in (1, 16, 4096, 65536, 300001, 300002):
        emx, emn = oracle.wedge(a, w)
        gmx, gmn = par_oracle.wedge(a, w, piece=12345)
        assert np.array_equal(gmx, emx) and np.array_equal(gmn, emn)


def test_batched_bands_envelopes_equal_one_call():
    rng = synth.rng_for("tests", 911)
    packed, offs, wins = synth.batched_series(S=60, lo=1, hi=5000, wlo=1, whi=700, rng=rng)
    eoo, emx, emn = oracle.batched(packed, offs, wins)
    goo, gmx, gmn = par_oracle.batched(packed, offs, wins)
    assert np.array_equal(goo, eoo) and np.array_equal(gmx, emx) and np.array_equal(gmn, emn)
    img = synth.gaussian_field(301, 157, sigma=3.0, rng=rng)
    for wr, wc in ((1, 1), (3, 5), (15, 15), (63, 9)):
        emx, emn = oracle.filter2d(img, wr, wc)
        gmx, gmn = par_oracle.filter2d(img, wr, wc, band=37)
        assert np.array_equal(gmx, emx) and np.array_equal(gmn, emn)
    for op in ("erode", "dilate", "open", "close"):
        assert np.array_equal(par_oracle.morph2d(img, op, 7, 3, band=29), oracle.morph2d(img, op, 7, 3))
    radii = rng.integers(0, 50, wins.size)
    eu, el = oracle.envelope_batched(packed, offs, radii)
    gu, gl = par_oracle.envelope_batched(packed, offs, radii)
    assert np.array_equal(gu, eu) and np.array_equal(gl, el)
