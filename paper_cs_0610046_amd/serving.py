"""Open-loop load generator for the serving engine (``maxmin_engine_*``).

Filter requests arrive as a Poisson process at ``rate`` per second: dtype
uniform over float32 / float64 / int32, length log-uniform in [256, 4 Mi],
window uniform in [2, 8192] (about a quarter have w > n and finish at once).
Alongside, ``n_streams`` persistent float32 streams (window 512) each push
``chunk``-sample chunks as a Poisson process at ``stream_rate`` per second;
their carries stay on the device.  Submission is done by the engine's C++
replay thread at the scheduled times; this module only prepares the
schedule, pinned payloads, and reads back latencies.

Payloads come from pinned pools (one 4 Mi-sample series per dtype, prefixes
of it serve every request), and requests of one dtype share pinned output
buffers: the benchmark measures timing, not values (the serving tests check
values with private buffers, up to the workload's own scale).  A request
refused by the engine's back-pressure (its admission queue is full) counts
as refused, not as a latency sample.
"""
import threading
import time

import numpy as np

from . import binding as mm
from . import synth

MAX_N = 4 << 20


def _pinned(arr):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(arr)).pin_memory()
    return t


def pcie_copy_rates(nbytes=1 << 30):
    """Achieved pinned host <-> device copy bandwidth (GB/s): host to
    device, device to host, and both at once on two streams."""
    import torch
    h1 = torch.empty(nbytes, dtype=torch.uint8).pin_memory()
    h2 = torch.empty(nbytes, dtype=torch.uint8).pin_memory()
    d1 = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    d2 = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()

    def timed(fn, reps=3):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps

    def both():
        with torch.cuda.stream(s1):
            d1.copy_(h1, non_blocking=True)
        with torch.cuda.stream(s2):
            h2.copy_(d2, non_blocking=True)

    t_h2d = timed(lambda: d1.copy_(h1, non_blocking=True))
    t_d2h = timed(lambda: h2.copy_(d2, non_blocking=True))
    t_both = timed(both)
    return {"h2d_GBs": round(nbytes / t_h2d / 1e9, 1), "d2h_GBs": round(nbytes / t_d2h / 1e9, 1),
            "both_ways_GBs": round(2 * nbytes / t_both / 1e9, 1), "bytes": nbytes}


def serving_run(rate, duration, n_streams=1000, stream_rate=10.0, chunk=4096, stream_w=512,
                budget=64 << 30, lanes=4, max_batch=256, seed=0, warmup=0.0):
    """Replay ``warmup + duration`` seconds of the load; latency
    percentiles and throughput count the requests that arrive after the
    warm-up (throughput: their input samples over the time from the end of
    the warm-up to the last completion)."""
    import torch
    rng = np.random.default_rng(np.random.SeedSequence([synth.SEED_ROOT, synth.WORKLOAD_IDS["serving"], 7, seed]))
    total_s = warmup + duration
    reqs = synth.serving_requests(rate, total_s, rng)
    arr = synth.stream_arrivals(n_streams, stream_rate, total_s, np.random.default_rng(seed + 1))
    pools = {np.dtype(np.float32): _pinned(synth.random_walk(MAX_N, np.float32, rng)),
             np.dtype(np.float64): _pinned(synth.random_walk(MAX_N, np.float64, rng)),
             np.dtype(np.int32): _pinned(synth.uniform_i32(MAX_N, rng))}
    outs = {d: (torch.empty(MAX_N, dtype=p.dtype).pin_memory(), torch.empty(MAX_N, dtype=p.dtype).pin_memory())
            for d, p in pools.items()}
    chunks = _pinned(synth.random_walk(64 * chunk, np.float32, rng))
    chunk_out = (torch.empty(chunk, dtype=torch.float32).pin_memory(),
                 torch.empty(chunk, dtype=torch.float32).pin_memory())

    eng = mm.MaxMinEngine(budget, lanes, max_batch)
    sids = [eng.open_stream(torch.float32, stream_w) for _ in range(n_streams)]
    ev = [(t, 0, i) for i, t in enumerate(r[0] for r in reqs)] + [(t, 1, s) for t, s in arr]
    ev.sort()
    cnt = len(ev)
    at_s = np.empty(cnt)
    kind = np.empty(cnt, np.int32)
    dtc = np.zeros(cnt, np.int32)
    nn = np.empty(cnt, np.int64)
    ww = np.zeros(cnt, np.int64)
    sid = np.zeros(cnt, np.int64)
    h_in = np.empty(cnt, np.uint64)
    h_mx = np.empty(cnt, np.uint64)
    h_mn = np.empty(cnt, np.uint64)
    for j, (t, k, i) in enumerate(ev):
        at_s[j] = t
        kind[j] = k
        if k == 0:
            _, d, n, w = reqs[i]
            dtc[j] = mm.dtype_code(d)
            nn[j], ww[j] = n, w
            h_in[j] = pools[d].data_ptr()
            h_mx[j], h_mn[j] = outs[d][0].data_ptr(), outs[d][1].data_ptr()
        else:
            sid[j] = sids[i]
            nn[j] = chunk
            h_in[j] = chunks.data_ptr() + 4 * chunk * (j % 64)
            h_mx[j], h_mn[j] = chunk_out[0].data_ptr(), chunk_out[1].data_ptr()

    results = []
    box = {}

    def go():
        box["ids"], box["lag"] = eng.replay(at_s.tolist(), kind.tolist(), dtc.tolist(), nn.tolist(), ww.tolist(),
                                            sid.tolist(), h_in.tolist(), h_mx.tolist(), h_mn.tolist())

    t0 = time.perf_counter()
    th = threading.Thread(target=go)
    th.start()
    while th.is_alive():
        results += eng.poll()
        time.sleep(0.01)
    th.join()
    eng.drain()
    results += eng.poll()
    wall = time.perf_counter() - t0 - warmup
    st = eng.stats()
    for s in sids:
        eng.close_stream(s)
    eng.close()

    ids = box["ids"]
    kind_of = dict(zip(ids, kind.tolist()))
    n_of = dict(zip(ids, nn.tolist()))
    at_of = dict(zip(ids, at_s.tolist()))
    measured = at_s >= warmup
    refused = int(sum(1 for i, m in zip(ids, measured) if m and i < 0))
    lat = {0: [], 1: []}
    bad = 0
    elems = 0
    for rid, no, l, status in results:
        if at_of[rid] < warmup:
            continue
        if status != 0:
            bad += 1
            continue
        lat[kind_of[rid]].append(l)
        elems += n_of[rid]

    def pct(v, q):
        return round(float(np.percentile(v, q)) * 1e3, 4) if v else None

    allv = lat[0] + lat[1]
    return {"rate_per_s": rate, "duration_s": duration, "warmup_s": warmup, "wall_s": round(wall, 3),
            "requests": int(((kind == 0) & measured).sum()), "pushes": int(((kind == 1) & measured).sum()),
            "failed": bad, "refused": refused,
            "p50_ms": pct(allv, 50), "p99_ms": pct(allv, 99),
            "filter_p50_ms": pct(lat[0], 50), "filter_p99_ms": pct(lat[0], 99),
            "push_p50_ms": pct(lat[1], 50), "push_p99_ms": pct(lat[1], 99),
            "gelem_s": round(elems / wall / 1e9, 3), "batches": st["batches"],
            "peak_budget_gb": round(st["peak_bytes"] / 1e9, 3),
            "max_submit_lag_ms": round(max(box["lag"]) * 1e3, 3) if box["lag"] else 0.0}
