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
values with private buffers).
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


def serving_run(rate, duration, n_streams=1000, stream_rate=10.0, chunk=4096, stream_w=512,
                budget=64 << 30, lanes=4, max_batch=256, seed=0):
    import torch
    rng = np.random.default_rng(np.random.SeedSequence([synth.SEED_ROOT, synth.WORKLOAD_IDS["serving"], 7, seed]))
    reqs = synth.serving_requests(rate, duration, rng)
    arr = synth.stream_arrivals(n_streams, stream_rate, duration, np.random.default_rng(seed + 1))
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
    wall = time.perf_counter() - t0
    st = eng.stats()
    for s in sids:
        eng.close_stream(s)
    eng.close()

    kind_of = dict(zip(box["ids"], kind.tolist()))
    n_of = dict(zip(box["ids"], nn.tolist()))
    lat = {0: [], 1: []}
    bad = 0
    elems = 0
    for rid, no, l, status in results:
        if status != 0:
            bad += 1
            continue
        lat[kind_of[rid]].append(l)
        elems += n_of[rid]

    def pct(v, q):
        return round(float(np.percentile(v, q)) * 1e3, 4) if v else None

    allv = lat[0] + lat[1]
    return {"rate_per_s": rate, "duration_s": duration, "wall_s": round(wall, 3), "requests": int((kind == 0).sum()),
            "pushes": int((kind == 1).sum()), "failed": bad,
            "p50_ms": pct(allv, 50), "p99_ms": pct(allv, 99),
            "filter_p50_ms": pct(lat[0], 50), "filter_p99_ms": pct(lat[0], 99),
            "push_p50_ms": pct(lat[1], 50), "push_p99_ms": pct(lat[1], 99),
            "gelem_s": round(elems / wall / 1e9, 3), "batches": st["batches"],
            "peak_budget_gb": round(st["peak_bytes"] / 1e9, 3),
            "max_submit_lag_ms": round(max(box["lag"]) * 1e3, 3) if box["lag"] else 0.0}
