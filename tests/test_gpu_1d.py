"""GPU parity of the 1-D filter (plain, stream, batched) against the CPU
oracle, bit-exact, through the C ABI.  Sizes span several tiles and ragged
tails; every strategy is forced on every shape it can handle."""
import numpy as np
import pytest

import oracle
from paper_cs_0610046_amd import binding as mm
from paper_cs_0610046_amd import synth
from gpu_util import assert_bits_equal, note, to_dev, to_host

pytestmark = pytest.mark.gpu

DTS = [np.float32, np.float64, np.int32, np.uint16]
WINDOWS = [1, 2, 3, 7, 8, 9, 16, 17, 63, 64, 65, 255, 256, 511, 512, 513, 1000, 1023, 1024, 1025, 2047, 2048,
           2049, 3000, 4096, 5000]


def gen(n, dt, rng, kind):
    if kind == "walk":
        a = synth.random_walk(n, np.float64, rng)
        if dt == np.int32:
            return np.round(a * 1000).astype(np.int32)
        if dt == np.uint16:
            return (np.round(a * 10).astype(np.int64) % 65536).astype(np.uint16)
        return a.astype(dt)
    if kind == "ties":
        return synth.small_alphabet(n, 5, dt, rng)
    if kind == "ramp":
        return np.arange(n).astype(dt) if dt != np.uint16 else (np.arange(n) % 65536).astype(np.uint16)
    raise ValueError(kind)


def run_filter(a, w, strategy=mm.STRATEGY_AUTO, offset=0):
    import torch
    mm.maxmin_set_strategy(strategy)
    try:
        buf = to_dev(np.concatenate([np.zeros(offset, a.dtype), a]))
        x = buf[offset:]
        mx, mn = mm.maxmin_filter(x, w)
        torch.cuda.synchronize()
        mm.maxmin_check_stream()
        return to_host(mx, a.dtype), to_host(mn, a.dtype)
    finally:
        mm.maxmin_set_strategy(mm.STRATEGY_AUTO)


def check(a, w, what, **kw):
    gmx, gmn = run_filter(a, w, **kw)
    omx, omn = oracle.wedge(a, w)
    assert_bits_equal(gmx, omx, what + " max")
    assert_bits_equal(gmn, omn, what + " min")


@pytest.mark.parametrize("dt", DTS, ids=lambda d: np.dtype(d).name)
def test_plain_all_windows(dt):
    rng = synth.rng_for("tests", 100)
    for w in WINDOWS:
        for n in sorted({w, w + 1, 2 * w + 3, 5000, 2048 + w - 1, 2049 + w - 1, 4096 + w + 7}):
            kind = ["walk", "ties", "ramp"][(n + w) % 3]
            a = gen(n, dt, rng, kind)
            note("plain dt=%s n=%d w=%d kind=%s" % (np.dtype(dt).name, n, w, kind))
            check(a, w, "n=%d w=%d %s" % (n, w, kind))


@pytest.mark.parametrize("strategy", [mm.STRATEGY_TILE, mm.STRATEGY_CHUNK, mm.STRATEGY_RUN], ids=["tile", "chunk", "run"])
def test_forced_strategies_agree(strategy):
    rng = synth.rng_for("tests", 101)
    for dt in DTS:
        for w in [1, 2, 5, 33, 100, 512, 700, 1024, 1025, 1500, 2048, 2049, 3000, 4096, 4097, 6144, 6145, 8192] + \
                 ([8193, 9000] if strategy != mm.STRATEGY_TILE else []):
            n = int(rng.integers(w, 3 * 2048 + w))
            a = gen(n, dt, rng, "walk" if w % 2 else "ties")
            note("forced=%d dt=%s n=%d w=%d" % (strategy, np.dtype(dt).name, n, w))
            check(a, w, "forced %d n=%d w=%d" % (strategy, n, w), strategy=strategy)


def test_small_and_degenerate():
    rng = synth.rng_for("tests", 102)
    for dt in DTS:
        for n, w in [(1, 1), (2, 1), (2, 2), (3, 2), (5, 5), (1, 2), (0, 1), (10, 11), (4097, 4097), (4098, 4097)]:
            a = gen(n, dt, rng, "walk")
            note("degenerate dt=%s n=%d w=%d" % (np.dtype(dt).name, n, w))
            check(a, w, "n=%d w=%d" % (n, w))


def test_misaligned_pointers():
    rng = synth.rng_for("tests", 103)
    for dt in DTS:
        for off in (1, 2, 3):
            for w in (7, 300, 2000):
                a = gen(7777, dt, rng, "walk")
                note("misaligned dt=%s off=%d w=%d" % (np.dtype(dt).name, off, w))
                check(a, w, "offset %d w=%d" % (off, w), offset=off)


def test_misaligned_outputs():
    """Input, max and min pointers at independent element offsets (each
    misalignment modulo 16 bytes, equal and unequal between the outputs),
    over several wavefronts, runs and a ragged tail."""
    import torch
    rng = synth.rng_for("tests", 107)
    for dt in DTS:
        tdt = to_dev(np.zeros(1, dt)).dtype
        for oi, ox, on in ((0, 1, 1), (1, 2, 2), (3, 1, 2), (5, 7, 7), (2, 0, 3), (7, 6, 0)):
            for w in (3, 300, 1000):
                n = 70001 + oi
                a = gen(n, dt, rng, "walk")
                buf = to_dev(np.concatenate([np.zeros(oi, dt), a]))
                no = n - w + 1
                bmx = torch.empty(no + 8, dtype=tdt, device="cuda")
                bmn = torch.empty(no + 8, dtype=tdt, device="cuda")
                note("misaligned-out dt=%s in=%d max=%d min=%d w=%d" % (np.dtype(dt).name, oi, ox, on, w))
                mm.maxmin_filter(buf[oi:], w, bmx[ox:ox + no], bmn[on:on + no])
                torch.cuda.synchronize()
                omx, omn = oracle.wedge(a, w)
                assert_bits_equal(to_host(bmx[ox:ox + no], dt), omx, "max offsets %d/%d/%d" % (oi, ox, on))
                assert_bits_equal(to_host(bmn[on:on + no], dt), omn, "min offsets %d/%d/%d" % (oi, ox, on))


@pytest.mark.parametrize("path", ["onepass", "onepass-now", "onepass-defer", "twopass", "lookback"])
@pytest.mark.parametrize("strategy", [mm.STRATEGY_AUTO, mm.STRATEGY_CHUNK, mm.STRATEGY_RUN], ids=["auto", "chunk", "run"])
def test_large_windows(strategy, path, monkeypatch):
    """Windows of more than one chunk: the one-pass column kernel (records
    between sibling workgroups; its outputs stored in the step of their
    records or, MAXMIN_LONG_DEFER=1, one step later -- by default from 32
    chunks per block), the two passes (MAXMIN_LONG_ONEPASS=0: aggregates,
    then columns) and the look-back chunk kernel (MAXMIN_LONG_LOOKBACK=1);
    every dtype, block counts from one to dozens with a ragged last block,
    and a window longer than 256 chunks."""
    lookback = "1" if path == "lookback" else "0"
    monkeypatch.setenv("MAXMIN_LONG_LOOKBACK", lookback)
    monkeypatch.setenv("MAXMIN_LONG_ONEPASS", "0" if path == "twopass" else "1")
    if path == "onepass":
        monkeypatch.delenv("MAXMIN_LONG_DEFER", raising=False)
    else:
        monkeypatch.setenv("MAXMIN_LONG_DEFER", "1" if path == "onepass-defer" else "0")
    rng = synth.rng_for("tests", 104)
    a = gen(300000, np.float32, rng, "walk")
    for w in (2048, 4096, 4100, 65536, 100000, 299999, 300000):
        note("large-w n=300000 w=%d strategy=%d lookback=%s" % (w, strategy, lookback))
        check(a, w, "w=%d" % w, strategy=strategy)
    if strategy == mm.STRATEGY_AUTO:
        for dt in DTS:
            # 10000 and 65536: the two-pass kernels with 2048-element chunks
            for w, n in ((4097, 4097), (4097, 3 * 4097 + 5), (8192, 8192 * 7 + 4095), (10000, 10000 * 6 + 123),
                         (12289, 12289 * 5 + 1), (20000, 20000 * 30 + 19999), (65536, 65536 * 3 + 5),
                         (1 << 20, (1 << 20) + 77)):
                b = gen(n, dt, rng, "walk" if w % 2 else "ties")
                note("large-w dt=%s n=%d w=%d lookback=%s" % (np.dtype(dt).name, n, w, lookback))
                check(b, w, "dt=%s n=%d w=%d" % (np.dtype(dt).name, n, w))


@pytest.mark.parametrize("ranges", ["0", "8", "16", "32"])
def test_chunk_ticket_ranges(ranges, monkeypatch):
    """The chunks of a series split into per-XCD ticket ranges (one-chunk
    windows 1024 < w <= 4096, and longer windows whose ranges first redo the
    chunks just before them); every range count gives the oracle's bits,
    with chunk counts that do not divide evenly into the ranges."""
    monkeypatch.setenv("MAXMIN_CHUNK_RANGES", ranges)
    monkeypatch.setenv("MAXMIN_CHUNK_RANGES_LONG", ranges)
    monkeypatch.setenv("MAXMIN_LONG_LOOKBACK", "1")  # ranges belong to the look-back kernel
    rng = synth.rng_for("tests", 106)
    for dt in (np.float32, np.float64):
        for w, n in ((1025, 1100003), (1500, 1500 * 700 + 311), (4096, 4096 * 1031 + 4095),
                     (5000, 2500 * 1400 + 77), (9000, 3000 * 1500 + 1234), (65536, 4096 * 1100 + 999)):
            a = gen(n, dt, rng, "walk")
            note("ranges=%s dt=%s n=%d w=%d" % (ranges, np.dtype(dt).name, n, w))
            check(a, w, "ranges=%s n=%d w=%d" % (ranges, n, w), strategy=mm.STRATEGY_CHUNK)


@pytest.mark.parametrize("run", [None, "2048", "4096", "10000"])
def test_tile_windows_over_two_subtiles(run, monkeypatch):
    """2048 < w <= 8192: the tile kernel with blocks of a whole sub-tile,
    whose windows end two, three or four sub-tiles after they start (the
    whole sub-tiles between from their totals).  Runs of one, two and four
    sub-tiles (so every run boundary re-reads a halo of up to four
    sub-tiles), n from a single window to several runs with a ragged tail,
    ties and ramps, misaligned input and outputs, max-only and min-only."""
    import torch
    if run is not None:
        monkeypatch.setenv("MAXMIN_TILE_RUN", run)
    rng = synth.rng_for("tests", 108)
    for dt in DTS:
        tdt = to_dev(np.zeros(1, dt)).dtype
        for w in (2049, 2050, 2304, 3000, 4095, 4096, 4097, 5000, 6144, 6145, 7777, 8192):
            assert mm.maxmin_plan(dt, 1 << 20, w) == mm.STRATEGY_TILE
            for n in sorted({w, w + 1, w + 2047, w + 2048, w + 4095, 3 * 2048 + w + 5, 9 * 2048 + 13}):
                kind = ["walk", "ties", "ramp"][(n + w) % 3]
                a = gen(n, dt, rng, kind)
                note("tile2 run=%s dt=%s n=%d w=%d kind=%s" % (run, np.dtype(dt).name, n, w, kind))
                check(a, w, "tile2 n=%d w=%d %s" % (n, w, kind))
        # misaligned input and outputs; one output only
        for w in (3001, 5001, 7001):
            n = 40000 + 3
            a = gen(n, dt, rng, "walk")
            omx, omn = oracle.wedge(a, w)
            no = n - w + 1
            for oi, ox, on in ((1, 3, 2), (2, 0, 0)):
                buf = to_dev(np.concatenate([np.zeros(oi, dt), a]))
                bmx = torch.empty(no + 8, dtype=tdt, device="cuda")
                bmn = torch.empty(no + 8, dtype=tdt, device="cuda")
                note("tile2 misaligned run=%s dt=%s in=%d max=%d min=%d" % (run, np.dtype(dt).name, oi, ox, on))
                mm.maxmin_filter(buf[oi:], w, bmx[ox:ox + no], bmn[on:on + no])
                torch.cuda.synchronize()
                assert_bits_equal(to_host(bmx[ox:ox + no], dt), omx, "tile2 max offsets %d/%d/%d" % (oi, ox, on))
                assert_bits_equal(to_host(bmn[on:on + no], dt), omn, "tile2 min offsets %d/%d/%d" % (oi, ox, on))
            x = to_dev(a)
            note("tile2 one output run=%s dt=%s" % (run, np.dtype(dt).name))
            gmx, none = mm.maxmin_filter(x, w, which="max")
            none2, gmn = mm.maxmin_filter(x, w, which="min")
            assert none is None and none2 is None
            torch.cuda.synchronize()
            assert_bits_equal(to_host(gmx, dt), omx, "tile2 max-only")
            assert_bits_equal(to_host(gmn, dt), omn, "tile2 min-only")


def test_repeatable_bits():
    import torch
    rng = synth.rng_for("tests", 105)
    a = gen(1 << 18, np.float32, rng, "walk")
    x = to_dev(a)
    for w in (64, 4096):
        note("repeat w=%d" % w)
        r0 = [t.clone() for t in mm.maxmin_filter(x, w)]
        for _ in range(5):
            r = mm.maxmin_filter(x, w)
            torch.cuda.synchronize()
            assert torch.equal(r[0], r0[0]) and torch.equal(r[1], r0[1])


@pytest.mark.parametrize("w", [1, 2, 64, 512, 1024, 1025, 3000, 5000, 7000, 9000, 20000, 40000, 65536])
def test_stream_chunks_equal_one_shot(w, monkeypatch):
    """Every dtype.  w = 9000 and 65536 take the one-pass kernel (2048- and
    4096-element chunks), w = 40000 the two passes (forced; 4096-element
    chunks, k_chunk_col<T, 16>), w = 20000 the look-back chunk kernel
    (forced)."""
    if w == 20000:
        monkeypatch.setenv("MAXMIN_LONG_LOOKBACK", "1")
    if w == 40000:
        monkeypatch.setenv("MAXMIN_LONG_ONEPASS", "0")
    import torch
    rng = synth.rng_for("tests", 106)
    for dt in DTS:
        a = gen(40000 if w < 40000 else 300000, dt, rng, "walk")
        st = mm.maxmin_stream_create(to_dev(a[:1]).dtype, w)
        ost = oracle.Stream(dt, w)
        pos = 0
        outs = []
        while pos < a.size:
            m = int(rng.integers(0, 3 * w + 50))
            chunk = a[pos:pos + m]
            note("stream dt=%s w=%d pos=%d m=%d" % (np.dtype(dt).name, w, pos, m))
            gmx, gmn = st.push(to_dev(chunk))
            omx, omn = ost.push(chunk)
            torch.cuda.synchronize()
            assert_bits_equal(to_host(gmx, dt), omx, "stream max pos=%d" % pos)
            assert_bits_equal(to_host(gmn, dt), omn, "stream min pos=%d" % pos)
            outs.append(omx)
            pos += m
        assert st.samples == a.size
        st.close()
        mm.maxmin_check_stream()


@pytest.mark.parametrize("w", [1, 5, 64, 3000, 20000])
def test_stream_export_import(w):
    """Checkpoint and resume: at random points the GPU stream's state (t and
    its last min(t, w-1) samples) is exported, compared bit for bit with the
    oracle's, and a new handle is imported from it (alternately from the
    GPU's export and from the oracle's); the outputs continue exactly as
    the oracle stream's."""
    import torch
    rng = synth.rng_for("tests", 110)
    for dt in DTS:
        a = gen(60000, dt, rng, "walk")
        st = mm.maxmin_stream_create(to_dev(a[:1]).dtype, w)
        ost = oracle.Stream(dt, w)
        pos, k = 0, 0
        while pos < a.size:
            m = int(rng.integers(0, 2 * w + 40))
            chunk = a[pos:pos + m]
            note("stream export/import dt=%s w=%d pos=%d m=%d" % (np.dtype(dt).name, w, pos, m))
            gmx, gmn = st.push(to_dev(chunk))
            omx, omn = ost.push(chunk)
            torch.cuda.synchronize()
            assert_bits_equal(to_host(gmx, dt), omx, "stream max pos=%d" % pos)
            assert_bits_equal(to_host(gmn, dt), omn, "stream min pos=%d" % pos)
            pos += len(chunk)
            if rng.random() < 0.3:
                gt, gc = st.export()
                ot, oc = ost.export()
                assert gt == ot == pos
                assert_bits_equal(gc, oc, "exported carry at t=%d" % pos)
                st.close()
                k += 1
                st = mm.maxmin_stream_import(to_dev(a[:1]).dtype, w, *((gt, gc) if k % 2 else (ot, oc)))
                assert st.samples == pos
        st.close()
        mm.maxmin_check_stream()


def test_batched_mixed():
    import torch
    rng = synth.rng_for("tests", 107)
    for dt in DTS:
        S = 300
        lens = np.floor(np.exp(rng.uniform(np.log(1), np.log(30000), S))).astype(np.int64)
        lens[::17] = 0
        wins = rng.integers(1, 1100, S).astype(np.int64)
        wins[::7] = rng.integers(1025, 9000, wins[::7].size)
        wins[5] = lens[5] + 1
        offs = np.zeros(S + 1, np.int64)
        np.cumsum(lens, out=offs[1:])
        packed = gen(int(offs[-1]), dt, rng, "walk")
        oo = mm.maxmin_out_offsets(offs, wins)
        note("batched dt=%s S=%d total=%d" % (np.dtype(dt).name, S, offs[-1]))
        d_off, d_w, d_oo = (torch.from_numpy(v).cuda() for v in (offs, wins, oo))
        dmx, dmn = mm.maxmin_filter_batched(to_dev(packed), d_off, d_w, d_oo)
        torch.cuda.synchronize()
        mm.maxmin_check_stream()
        eoo, emx, emn = oracle.batched(packed, offs, wins)
        assert np.array_equal(oo, eoo)
        assert_bits_equal(to_host(dmx, dt), emx, "batched max")
        assert_bits_equal(to_host(dmn, dt), emn, "batched min")


def test_batched_graph_replay_matches_eager():
    """The batched call replays a captured graph on repeats; every replay,
    with eager work in between, gives the eager result."""
    import torch
    rng = synth.rng_for("tests", 108)
    packed, offs, wins = synth.batched_series(S=200, lo=10, hi=20000, wlo=1, whi=3000, rng=rng)
    oo = mm.maxmin_out_offsets(offs, wins)
    x = to_dev(packed)
    d_off, d_w, d_oo = (torch.from_numpy(v).cuda() for v in (offs, wins, oo))
    total = int(oo[-1])
    eoo, emx, emn = oracle.batched(packed, offs, wins)
    outs = (torch.empty(total, device="cuda"), torch.empty(total, device="cuda"))
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        for rep in range(4):
            note("batched graph replay %d" % rep)
            outs[0].fill_(0)
            outs[1].fill_(0)
            mm.maxmin_filter_batched(x, d_off, d_w, d_oo, outs[0], outs[1])
            y = mm.maxmin_filter(x[:5000], 33)  # eager work between replays
            s.synchronize()
            assert_bits_equal(to_host(outs[0], np.float32), emx, "replay %d max" % rep)
            assert_bits_equal(to_host(outs[1], np.float32), emn, "replay %d min" % rep)
            del y
    mm.maxmin_check_stream(s)


@pytest.mark.parametrize("plan", ["tile", "chunk"])
@pytest.mark.parametrize("run", ["1", "2", "4"])
def test_batched_plans(plan, run, monkeypatch):
    """Every batched plan the autotuner can choose gives the oracle's bits:
    all size classes on the tile kernel of their lag or on the chunk
    kernel, batched tiles of 1, 2 and 4 sub-tiles; series at any element
    offset, lengths across 2^16 and 2^20, windows to 12000, empty series
    and w > n."""
    import torch
    monkeypatch.setenv("MAXMIN_BATCH_PLAN", plan)
    monkeypatch.setenv("MAXMIN_BATCH_RUN", run)
    rng = synth.rng_for("tests", 109)
    for dt in (np.float32, np.float64, np.uint16):
        S = 60
        lens = np.floor(np.exp(rng.uniform(0, np.log(80000), S))).astype(np.int64)
        lens[:4] = [(1 << 20) + 3, 70001, 0, 5]
        wins = rng.integers(1, 2100, S).astype(np.int64)
        wins[::3] = rng.integers(2049, 12000, wins[::3].size)
        wins[3] = 9
        offs = np.zeros(S + 1, np.int64)
        np.cumsum(lens, out=offs[1:])
        packed = gen(int(offs[-1]), dt, rng, "walk")
        oo = mm.maxmin_out_offsets(offs, wins)
        note("batched plan=%s run=%s dt=%s total=%d" % (plan, run, np.dtype(dt).name, offs[-1]))
        d_off, d_w, d_oo = (torch.from_numpy(v).cuda() for v in (offs, wins, oo))
        dmx, dmn = mm.maxmin_filter_batched(to_dev(packed), d_off, d_w, d_oo)
        torch.cuda.synchronize()
        mm.maxmin_check_stream()
        _, emx, emn = oracle.batched(packed, offs, wins)
        assert_bits_equal(to_host(dmx, dt), emx, "batched plan=%s run=%s max" % (plan, run))
        assert_bits_equal(to_host(dmn, dt), emn, "batched plan=%s run=%s min" % (plan, run))
