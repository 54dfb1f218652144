"""Benchmark of the MI355X running max-min filter (one GPU).

A step is one pass of the hot path over the n = 2**28 float32 random-walk
series: the running max and min at each of the windows 16, 256, 4096 and
65536 (the tile kernel serves the first three -- its instantiation for
windows over one sub-tile at w = 4096 -- and the two chunk passes, chunk
aggregates then columns of chunks, the last).  ``value`` is input elements
processed per second over the K timed steps (Gelem/s), inputs already
resident in HBM.

Also reported on the same JSON line (not part of ``value``):
* ``per_window``   -- each window's launch time, Gelem/s and % of 8 TB/s
  (algorithmic bytes: n*s read + 2*(n-w+1)*s written) and of the measured
  copy ceiling,
* ``roofline``     -- the dominant kernel (most time per step) against HBM
  peak and against the measured copy ceiling, with its measured HBM traffic
  per launch when the committed counter summary matches the current kernel
  sources,
* ``ceiling``      -- the device's practical HBM ceiling: a 4 GiB device copy
  and fill (``--ceiling`` runs only this),
* ``large_other``  -- the rest of the n = 2**28 workload: float32 piecewise
  monotone and ramp, the float64 copy of the walk, int32 uniform,
* ``plain``        -- n = 2**20 float32, w = 64 (latency-bound),
* ``batched``      -- 10,000 float32 random walks, lengths log-uniform in
  [1e3, 1e6], windows uniform in [2, 1024], one batched call (graph replay),
* ``image``        -- 8192 x 8192 float32 (``image_u16``: uint16), w x w windows,
  one fused pass or rows then columns (the ``path`` field),
* ``argfilter``    -- n = 2**28 float32 walk, values plus leftmost locations,
* ``max_only``     -- the same walk, w = 256, only the max output,
* ``envelope``     -- centered envelopes of 100,000 walks of 1024 samples,
* ``morphology``   -- opening of the 8192 x 8192 field with a 15 x 15 square,
* ``cpu_baseline`` -- the CPU oracle (single thread) on a bounded sample, with
  the host's CPU model and core counts; ``batched.cpu_oracle_parallel`` is
  the oracle over the batch's series on up to 16 host threads.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
WINDOWS = (16, 256, 4096, 65536)
SERVING_RATES = "1000,4000,16000"
SERVING_SECONDS = 30.0
SERVING_WARMUP = 3.0


def alg_bytes(n, w, s):
    return n * s + 2 * max(0, n - w + 1) * s


def kernel_name(strategy, w):
    """The kernel rocprofv3 names for a single-series float32 launch: the
    tile kernel (last template argument: how many sub-tiles after its start
    a window may end), or for w > 8192 the one-pass long-window kernel
    (columns of 4096-element chunks; 8 elements per thread when a window
    spans at most three chunks, else 16; outputs one step behind the
    records from 32 chunks per block on)."""
    if strategy == "tile":
        return "mm::k_tile<0, float, false, %d>" % (1 if w <= 2048 else (w + 2047) // 2048)
    k = (w + 4095) // 4096
    v = 8 if k <= 3 else 16
    chunks = (w + 256 * v - 1) // (256 * v)
    return "mm::k_chunk_col1<float, %d, %s>" % (v, "true" if chunks >= 32 else "false")


# Sources whose change invalidates counter-derived traffic figures.
KERNEL_SOURCES = ("paper_cs_0610046_amd/csrc/mm_kernels_1d.hip", "paper_cs_0610046_amd/csrc/mm_device.hpp",
                  "paper_cs_0610046_amd/csrc/mm_launch.hpp", "paper_cs_0610046_amd/csrc/mm_abi.cpp")
TRAFFIC_FILE = "profiles/hbm_traffic_f32_walk_n2p28.md"


def kernel_source_hash():
    """Hash of the kernel sources' code: comments and whitespace are dropped,
    so editing documentation does not void the counter figures."""
    import hashlib
    import re
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f)) as fh:
            text = fh.read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()[:16]


def measured_traffic(kernel, n):
    """HBM bytes per launch of ``kernel`` from the committed counter summary,
    or None when it is missing, for another size, or older than the kernel
    sources (its recorded source hash differs)."""
    path = os.path.join(ROOT, TRAFFIC_FILE)
    if n != 1 << 28 or not os.path.exists(path):
        return None, "none"
    vals, src = {}, None
    for line in open(path):
        line = line.strip()
        if line.startswith("source-hash:"):
            src = line.split(":", 1)[1].strip()
        elif line.startswith("traffic-per-launch:"):
            k, v = line.split(":", 1)[1].rsplit("=", 1)
            vals[k.strip()] = float(v)
    if src != kernel_source_hash():
        return None, "stale (kernel sources changed since the counters were taken)"
    if kernel not in vals:
        return None, "none"
    return vals[kernel], TRAFFIC_FILE


def measure_ceiling(torch, dev, stream, gib=4, iters=10):
    """Practical HBM ceiling on this device: a device-to-device copy of
    ``gib`` GiB (each byte read once and written once) and a fill of the
    same buffer (written once), both far larger than the last-level cache,
    timed with events on the launch stream (median of ``iters``)."""
    nbytes = gib << 30
    src = torch.empty(nbytes // 4, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    src.fill_(1.0)
    dst.copy_(src)
    torch.cuda.synchronize()
    tc = float(np.median(timed(lambda: dst.copy_(src), iters, stream)))
    tf = float(np.median(timed(lambda: dst.fill_(2.0), iters, stream)))
    del src, dst
    return {"copy_GBs": round(2 * nbytes / (tc * 1e-3) / 1e9, 1), "copy_ms": round(tc, 4),
            "fill_GBs": round(nbytes / (tf * 1e-3) / 1e9, 1), "fill_ms": round(tf, 4),
            "buffer_bytes": nbytes,
            "what": "torch device copy (read + write) and fill (write) of %d GiB float32 buffers, median of %d "
                    "event-timed calls" % (gib, iters)}


def host_cpu():
    """Host CPU model and core counts (for the CPU baseline)."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count() or 1
    return {"model": model, "logical_cpus": os.cpu_count(), "usable_cpus": usable}


def timed(fn, iters, stream):
    import torch
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(iters)]
    for a, b in evs:
        a.record(stream)
        fn()
        b.record(stream)
    torch.cuda.synchronize()
    return [a.elapsed_time(b) for a, b in evs]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n-log2", type=int, default=28)
    ap.add_argument("--extras", type=int, default=1, help="also run plain / batched / image workloads")
    ap.add_argument("--cpu-sample-log2", type=int, default=26)
    ap.add_argument("--autotune", type=int, default=1, help="measure the planner's launch parameters first")
    ap.add_argument("--calib-copy", action="store_true",
                    help="run one 256 MiB device copy first (a known-size kernel for counter calibration)")
    ap.add_argument("--serving-rates", default=SERVING_RATES,
                    help="request rates (per s) of the serving runs, comma-separated ('none': no serving runs)")
    ap.add_argument("--serving-seconds", type=float, default=SERVING_SECONDS, help="measured seconds per rate")
    ap.add_argument("--serving-warmup", type=float, default=SERVING_WARMUP, help="warm-up seconds per rate")
    ap.add_argument("--serving-only", action="store_true", help="run only the serving sweep and print it")
    ap.add_argument("--ceiling", action="store_true",
                    help="only measure the device's copy / fill bandwidth (4 GiB buffers) and print it")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: the benchmark runs on one GPU; --gpus %d is not supported" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_cs_0610046_amd import binding as mm
    from paper_cs_0610046_amd import synth

    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    if args.calib_copy:
        src = torch.ones(64 << 20, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if args.ceiling:
        print(json.dumps({"ceiling": measure_ceiling(torch, dev, stream)}), flush=True)
        return
    if args.serving_only:
        print(json.dumps({"serving": run_serving(args)}), flush=True)
        return
    tuning = mm.maxmin_tuning(torch.float32)
    if args.autotune:
        t0 = time.time()
        tuning = mm.maxmin_autotune(torch.float32, 1 << 28)
        print("[bench] autotune %.2fs: %s" % (time.time() - t0, tuning), file=sys.stderr, flush=True)
    n = 1 << args.n_log2
    t0 = time.time()
    a = synth.random_walk(n, np.float32, synth.rng_for("large", 0))
    print("[bench] generated n=2^%d walk in %.1fs" % (args.n_log2, time.time() - t0), file=sys.stderr, flush=True)
    x = torch.from_numpy(a).to(dev)
    outs = {w: (torch.empty(n - w + 1, dtype=torch.float32, device=dev),
                torch.empty(n - w + 1, dtype=torch.float32, device=dev)) for w in WINDOWS}

    def step():
        for w in WINDOWS:
            mm.maxmin_filter(x, w, outs[w][0], outs[w][1])

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    mm.maxmin_check_stream()
    # per-launch timing with events on the launch stream (inside the timed steps)
    ev = {w: [] for w in WINDOWS}
    marks = []
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for _ in range(args.steps):
        for w in WINDOWS:
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            mm.maxmin_filter(x, w, outs[w][0], outs[w][1])
            e1.record(stream)
            marks.append((w, e0, e1))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    for w, e0, e1 in marks:
        ev[w].append(e0.elapsed_time(e1))
    mm.maxmin_check_stream()
    ms_per_step = wall * 1e3 / args.steps
    value = len(WINDOWS) * n / (wall / args.steps) / 1e9
    per_window = {}
    for w in WINDOWS:
        ms = float(np.mean(ev[w]))
        gb = alg_bytes(n, w, 4) / (ms * 1e-3) / 1e9
        per_window[str(w)] = {"ms": round(ms, 4), "gelem_s": round(n / (ms * 1e-3) / 1e9, 2),
                              "alg_GBs": round(gb, 1), "pct_hbm": round(100 * gb / HBM_PEAK_GBS, 1),
                              "strategy": "tile" if mm.maxmin_plan(torch.float32, n, w) == 1 else "chunk"}
    # the dominant kernel: the one with the most time per step; its roofline
    # point is its algorithmic bytes over its launches / their total time
    kern = {}
    for w in WINDOWS:
        k = kernel_name(per_window[str(w)]["strategy"], w)
        kern.setdefault(k, []).append(w)
    dom = max(kern, key=lambda k: sum(np.mean(ev[w]) for w in kern[k]))
    dom_ms = float(np.mean([t for w in kern[dom] for t in ev[w]]))
    dom_bytes = float(np.mean([alg_bytes(n, w, 4) for w in kern[dom]]))
    achieved = dom_bytes / (dom_ms * 1e-3) / 1e9
    traffic, tsrc = measured_traffic(dom, n)
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": None if traffic is None else int(round(traffic)),
                "traffic_unit": "bytes per launch (HBM, calibrated FETCH_SIZE + WRITE_SIZE)",
                "traffic_vs_alg": None if traffic is None else round(traffic / dom_bytes, 4),
                "traffic_source": tsrc,
                "kernel": dom, "windows": kern[dom], "alg_bytes_per_launch": int(dom_bytes),
                "avg_launch_ms": round(dom_ms, 4)}
    print("[bench] headline %.1f Gelem/s, %.3f ms/step" % (value, ms_per_step), file=sys.stderr, flush=True)
    del outs
    ceiling = measure_ceiling(torch, dev, stream)
    cgb = ceiling["copy_GBs"]
    for w in WINDOWS:
        per_window[str(w)]["pct_copy_ceiling"] = round(100 * per_window[str(w)]["alg_GBs"] / cgb, 1)
    roofline["frac_of_copy_ceiling"] = round(achieved / cgb, 4)
    print("[bench] ceiling copy %.0f GB/s fill %.0f GB/s" % (cgb, ceiling["fill_GBs"]), file=sys.stderr, flush=True)

    extras = {}
    if args.extras:
        extras = run_extras(torch, mm, synth, dev, stream, cgb)
        if args.serving_rates != "none":
            extras["serving"] = run_serving(args)

    # CPU oracle on a bounded sample of the same workload (rank 0, N=1 only)
    import oracle
    m = min(n, 1 << args.cpu_sample_log2)
    # one core, as the paper's single-threaded runs (restored afterwards)
    aff = os.sched_getaffinity(0)
    try:
        os.sched_setaffinity(0, {min(aff)})
    except OSError:
        pass
    t0 = time.perf_counter()
    for w in WINDOWS:
        oracle.wedge(a[:m], w)
    ct = time.perf_counter() - t0
    try:
        os.sched_setaffinity(0, aff)
    except OSError:
        pass
    cpu = {"value": round(len(WINDOWS) * m / ct / 1e9, 5), "unit": "Gelem/s", "cores": 1, "kind": "oracle",
           "sample": "first 2^%d elements of the same float32 walk, windows %s, one thread pinned to one core (g++ -O2 "
                     "monotonic-wedge oracle), %.1f s" % (args.cpu_sample_log2, list(WINDOWS), ct),
           "host": host_cpu()}

    line = {"metric": "Gelem/s and % HBM peak, batched vs plain kernel; serving p50/p99 latency",
            "value": round(value, 2), "unit": "Gelem/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4), "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": "single float32 random walk n=2^%d, windows %s" % (args.n_log2, list(WINDOWS)),
                       "n": n, "windows": list(WINDOWS)},
            "per_window": per_window, "roofline": roofline, "ceiling": ceiling, "cpu_baseline": cpu,
            "tuning": tuning}
    line.update(extras)
    print(json.dumps(line), flush=True)


def batched_cpu_parallel(packed, offs, wins, target=1 << 29):
    """The CPU oracle on the batched workload, series in parallel on the
    host's cores (at most 16 threads: one GPU's share of the host), over the
    first series that hold about ``target`` elements."""
    from concurrent.futures import ThreadPoolExecutor
    import oracle
    k = int(np.searchsorted(offs, min(target, int(offs[-1])))) or 1
    threads = max(1, min(16, host_cpu()["usable_cpus"]))

    def run(i):
        oracle.wedge(packed[offs[i]:offs[i + 1]], int(wins[i]))

    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=threads) as ex:
        list(ex.map(run, range(k)))
    ct = time.perf_counter() - t0
    m = int(offs[k])
    return {"value": round(m / ct / 1e9, 4), "unit": "Gelem/s", "cores": threads, "kind": "oracle",
            "sample": "first %d of the 10,000 series (%d elements), one series per task on %d threads, %.1f s" %
                      (k, m, threads, ct)}


def run_extras(torch, mm, synth, dev, stream, copy_gbs):
    out = {}
    # the rest of the n = 2^28 single-series workload: the other float32
    # inputs, and the float64 and int32 copies (same windows; not in `value`)
    others = {}
    for key, make, tdt, s in (
            ("f32_piecewise_monotone", lambda: synth.large_series("pwm"), torch.float32, 4),
            ("f32_ramp", lambda: synth.large_series("ramp"), torch.float32, 4),
            ("f64_walk", lambda: synth.random_walk(1 << 28, np.float64, synth.rng_for("large", 0)), torch.float64, 8),
            ("i32_uniform", lambda: synth.large_series("i32"), torch.int32, 4)):
        t0 = time.time()
        h = make()
        xo = torch.from_numpy(h).to(dev)
        del h
        n = xo.numel()
        res = {}
        for w in WINDOWS:
            o1 = torch.empty(n - w + 1, dtype=tdt, device=dev)
            o2 = torch.empty_like(o1)
            for _ in range(2):
                mm.maxmin_filter(xo, w, o1, o2)
            ts = timed(lambda: mm.maxmin_filter(xo, w, o1, o2), 10, stream)
            ms = float(np.median(ts))
            gb = alg_bytes(n, w, s) / (ms * 1e-3) / 1e9
            res[str(w)] = {"ms": round(ms, 4), "gelem_s": round(n / (ms * 1e-3) / 1e9, 2),
                           "pct_hbm": round(100 * gb / HBM_PEAK_GBS, 1),
                           "pct_copy_ceiling": round(100 * gb / copy_gbs, 1)}
            del o1, o2
        mm.maxmin_check_stream()
        step_ms = sum(r["ms"] for r in res.values())
        others[key] = {"per_window": res, "step_ms": round(step_ms, 4),
                       "gelem_s": round(len(WINDOWS) * n / (step_ms * 1e-3) / 1e9, 2)}
        print("[bench] %s %.3f ms per step of 4 windows (%.1fs)" % (key, step_ms, time.time() - t0),
              file=sys.stderr, flush=True)
        del xo
    out["large_other"] = {"workload": "n=2^28 single series, windows %s: float32 piecewise monotone and ramp, "
                                      "float64 walk, int32 uniform (algorithmic bytes n*s + 2*(n-w+1)*s; "
                                      "median of 10 event-timed launches per window)" % list(WINDOWS),
                          "per_input": others}
    # plain: n = 2^20 float32 uniform, w = 64
    a = synth.uniform01(1 << 20)
    x = torch.from_numpy(a).to(dev)
    mx = torch.empty(x.numel() - 63, device=dev)
    mn = torch.empty_like(mx)
    for _ in range(5):
        mm.maxmin_filter(x, 64, mx, mn)
    ts = timed(lambda: mm.maxmin_filter(x, 64, mx, mn), 50, stream)
    ms = float(np.median(ts))
    # cold: 128 input/output sets (1.5 GiB) used in turn, so no call finds
    # its 4 MiB input in the 256 MB last-level cache
    sets = [(x.clone(), torch.empty_like(mx), torch.empty_like(mx)) for _ in range(128)]
    k = [0]

    def cold():
        xi, oi, pi = sets[k[0] % len(sets)]
        k[0] += 1
        mm.maxmin_filter(xi, 64, oi, pi)
    for _ in range(128):
        cold()
    ms_cold = float(np.median(timed(cold, 128, stream)))
    del sets
    # host time of one ABI call (enqueue only, no wait), over 2000 calls
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(2000):
        mm.maxmin_filter(x, 64, mx, mn)
    call_us = (time.perf_counter() - t0) / 2000 * 1e6
    torch.cuda.synchronize()
    out["plain"] = {"workload": "n=2^20 float32 uniform, w=64", "ms": round(ms, 4),
                    "gelem_s": round(x.numel() / (ms * 1e-3) / 1e9, 2),
                    "pct_hbm": round(100 * alg_bytes(x.numel(), 64, 4) / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 1),
                    "ms_cold": round(ms_cold, 4),
                    "pct_hbm_cold": round(100 * alg_bytes(x.numel(), 64, 4) / (ms_cold * 1e-3) / 1e9 / HBM_PEAK_GBS,
                                          1),
                    "abi_call_us": round(call_us, 2),
                    "note": "ms: event-timed call, input cache-resident; ms_cold: 128 buffer sets used in turn; "
                            "abi_call_us: host time to enqueue one call"}
    print("[bench] plain %.4f ms (cold %.4f ms, call %.1f us)" % (ms, ms_cold, call_us), file=sys.stderr, flush=True)
    del x, mx, mn

    # batched: 10,000 random walks, lengths log-uniform [1e3, 1e6], windows [2, 1024]
    t0 = time.time()
    packed, offs, wins = synth.batched_series()
    print("[bench] generated batched (%d elems) in %.1fs" % (packed.size, time.time() - t0), file=sys.stderr,
          flush=True)
    oo = mm.maxmin_out_offsets(offs, wins)
    xb = torch.from_numpy(packed).to(dev)
    cpu_par = batched_cpu_parallel(packed, offs, wins)
    del packed
    d_off, d_w, d_oo = (torch.from_numpy(v).to(dev) for v in (offs, wins, oo))
    total = int(oo[-1])
    bmx = torch.empty(total, device=dev)
    bmn = torch.empty(total, device=dev)
    s2 = torch.cuda.Stream(dev)
    with torch.cuda.stream(s2):
        for _ in range(3):
            mm.maxmin_filter_batched(xb, d_off, d_w, d_oo, bmx, bmn)
        ts = timed(lambda: mm.maxmin_filter_batched(xb, d_off, d_w, d_oo, bmx, bmn), 10, s2)
    mm.maxmin_check_stream(s2)
    ms = float(np.median(ts))
    N = int(offs[-1])
    ab = N * 4 + 2 * total * 4
    out["batched"] = {"workload": "10000 float32 walks, n log-uniform [1e3,1e6], w uniform [2,1024], graph replay",
                      "elements": N, "ms": round(ms, 4), "gelem_s": round(N / (ms * 1e-3) / 1e9, 2),
                      "pct_hbm": round(100 * ab / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 1),
                      "pct_copy_ceiling": round(100 * ab / (ms * 1e-3) / 1e9 / copy_gbs, 1),
                      "cpu_oracle_parallel": cpu_par}
    print("[bench] batched %.3f ms" % ms, file=sys.stderr, flush=True)
    del xb, bmx, bmn

    # image: 8192 x 8192, float32 Gaussian field and uint16 uniform, w x w
    for key, make, s in (("image", lambda: synth.gaussian_field(8192, 8192), 4),
                         ("image_u16", lambda: synth.uniform_u16((8192, 8192), synth.rng_for("image", 1)), 2)):
        img = make()
        if img.dtype == np.uint16:  # bit-for-bit through int16 (torch's uint16 has few ops)
            xi = torch.from_numpy(img.view(np.int16)).view(torch.uint16).to(dev)
        else:
            xi = torch.from_numpy(img).to(dev)
        del img
        res = {}
        for w in (3, 15, 63):
            o1 = torch.empty((8192 - w + 1, 8192 - w + 1), device=dev, dtype=xi.dtype)
            o2 = torch.empty_like(o1)
            for _ in range(2):
                mm.maxmin_filter_2d(xi, w, w, o1, o2)
            ts = timed(lambda: mm.maxmin_filter_2d(xi, w, w, o1, o2), 5, stream)
            ms = float(np.median(ts))
            ab = 8192 * 8192 * s + 2 * o1.numel() * s
            plan = mm.maxmin_plan_2d(xi.dtype, w, w)
            res[str(w)] = {"ms": round(ms, 4), "gelem_s": round(8192 * 8192 / (ms * 1e-3) / 1e9, 2),
                           "pct_hbm": round(100 * ab / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 1),
                           "path": "fused" if plan == mm.PLAN_2D_FUSED else "rows then columns"}
            del o1, o2
        out[key] = {"workload": "8192x8192 %s, w x w windows (algorithmic bytes: input + both outputs)" %
                    ("float32 Gaussian field + noise" if s == 4 else "uint16 uniform"), "per_window": res}
        print("[bench] %s done" % key, file=sys.stderr, flush=True)
        del xi

    # arg filter: n = 2^28 float32 walk, values and leftmost locations
    xa = torch.from_numpy(synth.random_walk(1 << 28, np.float32, synth.rng_for("large", 0))).to(dev)
    res = {}
    for w in (256, 4096, 65536):
        outs = mm.maxmin_argfilter(xa, w)
        mm.maxmin_argfilter(xa, w, *outs)
        ts = timed(lambda: mm.maxmin_argfilter(xa, w, *outs), 5, stream)
        ms = float(np.median(ts))
        ab = xa.numel() * 4 + outs[0].numel() * (2 * 4 + 2 * 8)
        res[str(w)] = {"ms": round(ms, 4), "gelem_s": round(xa.numel() / (ms * 1e-3) / 1e9, 2),
                       "pct_hbm": round(100 * ab / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 1),
                       "path": "tile with locations" if w <= 4096 else
                       "chunk aggregates + columns of chunks with locations"}
        del outs
    out["argfilter"] = {"workload": "n=2^28 float32 walk; max, min and their leftmost int64 locations "
                                    "(algorithmic bytes: 4 read + 24 written per window)", "per_window": res}
    print("[bench] argfilter done", file=sys.stderr, flush=True)
    del xa

    # max-only filter: n = 2^28 float32 walk, w = 256, min output not requested
    xm = torch.from_numpy(synth.random_walk(1 << 28, np.float32, synth.rng_for("large", 0))).to(dev)
    om = torch.empty(xm.numel() - 255, device=dev)
    mm.maxmin_filter(xm, 256, om, None, which="max")
    ts = timed(lambda: mm.maxmin_filter(xm, 256, om, None, which="max"), 5, stream)
    ms = float(np.median(ts))
    ab = xm.numel() * 4 + om.numel() * 4
    out["max_only"] = {"workload": "n=2^28 float32 walk, w=256, max output only (4 read + 4 written per window)",
                       "ms": round(ms, 4), "gelem_s": round(xm.numel() / (ms * 1e-3) / 1e9, 2),
                       "pct_hbm": round(100 * ab / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 1)}
    del xm, om

    # centered envelopes over a batch of candidates (time-warping bounds)
    S, L = 100000, 1024
    rng = synth.rng_for("envelope", 0)
    radii = rng.integers(10, 101, S).astype(np.int64)
    offs = np.arange(S + 1, dtype=np.int64) * L
    xe = torch.from_numpy(synth.random_walk(S * L, np.float32, rng)).to(dev)
    d_off, d_r = torch.from_numpy(offs).to(dev), torch.from_numpy(radii).to(dev)
    eu, el = torch.empty_like(xe), torch.empty_like(xe)
    for _ in range(2):
        mm.maxmin_envelope_batched(xe, d_off, d_r, eu, el)
    ts = timed(lambda: mm.maxmin_envelope_batched(xe, d_off, d_r, eu, el), 5, stream)
    ms = float(np.median(ts))
    ab = 3 * xe.numel() * 4
    out["envelope"] = {"workload": "100,000 float32 walks of 1024 samples, radius uniform [10, 100], one batched "
                                   "call (one wavefront per short series)",
                       "ms": round(ms, 4), "gelem_s": round(xe.numel() / (ms * 1e-3) / 1e9, 2),
                       "pct_hbm": round(100 * ab / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 1)}
    del xe, eu, el

    # morphology: opening of the 8192^2 float32 field with a 15 x 15 square
    img = synth.gaussian_field(8192, 8192)
    xi = torch.from_numpy(img).to(dev)
    del img
    oo = mm.maxmin_morph_2d(xi, "open", 15)
    ts = timed(lambda: mm.maxmin_morph_2d(xi, "open", 15, out=oo), 5, stream)
    ms = float(np.median(ts))
    ab = xi.numel() * 4 + oo.numel() * 4
    out["morphology"] = {"workload": "opening of the 8192x8192 float32 field, 15x15 square (erosion then dilation, "
                                     "each a one-output 2-D filter)", "ms": round(ms, 4),
                         "gelem_s": round(xi.numel() / (ms * 1e-3) / 1e9, 2),
                         "pct_hbm": round(100 * ab / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 1)}
    del xi, oo

    return out


def run_serving(args):
    """Poisson filter requests + 1000 persistent streams, 64 GB budget: per
    rate, a warm-up, then the measured seconds; and the achieved pinned
    PCIe copy rates that bound it."""
    from paper_cs_0610046_amd.serving import pcie_copy_rates, serving_run
    pcie = pcie_copy_rates()
    print("[bench] pcie %s" % pcie, file=sys.stderr, flush=True)
    srv = []
    for rate in [int(r) for r in args.serving_rates.split(",") if r]:
        r = serving_run(rate, args.serving_seconds, n_streams=1000, stream_rate=10.0, warmup=args.serving_warmup)
        srv.append(r)
        print("[bench] serving rate=%d p50=%s p99=%s ms %.3f Gelem/s refused=%d" % (
            rate, r["p50_ms"], r["p99_ms"], r["gelem_s"], r["refused"]), file=sys.stderr, flush=True)
    return {"workload": "Poisson filter requests (f32/f64/i32, n log-uniform [256, 4Mi], w uniform [2, 8192]) + "
                        "1000 float32 streams x 10 chunks/s of 4096 at w=512; 64 GB HBM budget, 4 lanes; latency = "
                        "submit to completion incl. PCIe transfers; %.0f s measured after %.0f s of warm-up per rate"
                        % (args.serving_seconds, args.serving_warmup),
            "pcie": pcie, "per_rate": srv}


if __name__ == "__main__":
    main()
