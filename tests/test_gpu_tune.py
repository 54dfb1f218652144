"""The autotuner measures the planner's launch parameters on the device and
keeps the fastest; whatever it picks, results stay bit-identical to the
oracle (plain calls across window classes, and a batched call)."""
import numpy as np
import pytest

import oracle
from paper_cs_0610046_amd import binding as mm
from paper_cs_0610046_amd import synth
from gpu_util import assert_bits_equal, note, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.mark.timeout(600)
def test_autotune_then_parity():
    import torch
    note("autotune float32 n=2^22")
    t = mm.maxmin_autotune(np.float32, 1 << 22)
    assert t["measured"]
    assert t["tile_run_subtiles"] in (2, 4, 8, 16, 32) and t["tile_run_subtiles_long"] in (16, 32, 64, 128)
    assert t["rows_run_subtiles"] in (8, 16, 32)
    assert t["chunk_ranges_one_chunk"] in (0, 8, 16, 32) and t["chunk_ranges_long"] in (0, 16)
    assert t["long_window_strategy"] in ("chunk", "run")
    assert t["batched_tile_subtiles"] in (1, 2, 4)
    assert len(t["batched_plan"]) == 9 and set(t["batched_plan"].values()) <= {"tile", "chunk"}
    rng = synth.rng_for("tests", 800)
    a = synth.random_walk(3_000_001, np.float32, rng)
    x = to_dev(a)
    for w in (16, 256, 1024, 3000, 4096, 65536):
        note("after autotune w=%d" % w)
        mx, mn = mm.maxmin_filter(x, w)
        torch.cuda.synchronize()
        mm.maxmin_check_stream()
        emx, emn = oracle.wedge(a, w)
        assert_bits_equal(to_host(mx, np.float32), emx, "max w=%d" % w)
        assert_bits_equal(to_host(mn, np.float32), emn, "min w=%d" % w)
    # every size class of the batched plan (windows up to 10000; lengths
    # across 2^16 and 2^20)
    lens = rng.integers(0, 50000, 80)
    lens[:6] = [70000, 300000, 1 << 20, (1 << 20) + 5, 90000, 20000]
    wins = rng.integers(1, 2000, 80).astype(np.int64)
    wins[::4] = rng.integers(2049, 10000, wins[::4].size)
    offs = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    packed = synth.random_walk(int(offs[-1]), np.float32, rng)
    oo = mm.maxmin_out_offsets(offs, wins)
    d_off, d_w, d_oo = (torch.from_numpy(v).cuda() for v in (offs, wins, oo))
    note("after autotune batched")
    gmx, gmn = mm.maxmin_filter_batched(to_dev(packed), d_off, d_w, d_oo)
    torch.cuda.synchronize()
    _, emx, emn = oracle.batched(packed, offs, wins)
    assert_bits_equal(to_host(gmx, np.float32), emx, "batched max")
    assert_bits_equal(to_host(gmn, np.float32), emn, "batched min")
