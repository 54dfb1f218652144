"""Seeded synthetic inputs for the running max-min filter.

This module only draws numbers: it holds none of the filter's arithmetic, and
both the GPU tests/benchmark and the CPU oracle's tests take their inputs from
it.  Every generator is deterministic in its seed.

Seeds are ``numpy.random.SeedSequence([610046, workload_id, variant])``.

Float outputs are canonical for bit-exact selection: finite, no negative
zero, no subnormals (max/min of values that compare equal but differ in bits,
+0.0 and -0.0, would otherwise make the selected bit pattern depend on the
order of comparisons).

The workloads stand in for the paper's experiments (Section 5: i.i.d. noise and
a sine wave, a million points each) at the sizes this library targets:

* ``plain``      -- n = 2**20 float32 i.i.d. uniform [0, 1), w = 64.
* ``large``      -- n = 2**28: (a) random walk (cumulative sum of N(0,1)
  steps, accumulated in float64, then cast), (b) piecewise monotone
  (alternating up/down runs with geometric lengths of mean 100 and
  exponential step sizes), (c) strictly increasing float32 ramp; plus a
  float64 copy of (a) and an int32 i.i.d. uniform series over the full range.
* ``image``      -- 8192 x 8192: float32 smooth Gaussian random field
  (periodic Gaussian blur of white noise, sigma 16 px, unit std) plus
  0.25 * U[0, 1); uint16 i.i.d. uniform.
* ``batched``    -- 10,000 float32 random walks, lengths log-uniform in
  [1e3, 1e6], windows uniform in [2, 1024], packed with int64 offsets.
* ``serving``    -- Poisson request stream (see :func:`serving_requests`).
"""
import numpy as np

SEED_ROOT = 610046

WORKLOAD_IDS = {"plain": 1, "large": 2, "image": 3, "batched": 4, "serving": 5, "envelope": 6,
                "tests": 9}


def rng_for(workload, variant=0):
    wid = WORKLOAD_IDS[workload] if isinstance(workload, str) else int(workload)
    return np.random.default_rng(np.random.SeedSequence([SEED_ROOT, wid, int(variant)]))


def canonical(x):
    """Make a float array safe for bit-exact selection (in place): -0.0 -> +0.0,
    subnormals -> +0.0; raises on NaN/Inf.  Integer arrays pass through."""
    if x.dtype.kind != "f":
        return x
    if not np.all(np.isfinite(x)):
        raise ValueError("non-finite values in synthetic input")
    tiny = np.finfo(x.dtype).tiny
    x[np.abs(x) < tiny] = 0
    x += x.dtype.type(0.0)  # -0.0 + 0.0 == +0.0 in round-to-nearest
    return x


def check_canonical(x):
    if x.dtype.kind != "f":
        return True
    if not np.all(np.isfinite(x)):
        return False
    tiny = np.finfo(x.dtype).tiny
    nz = x != 0
    if np.any(np.abs(x[nz]) < tiny):
        return False
    return not np.any(np.signbit(x[~nz]))


# ---------------------------------------------------------------- 1-D series
def uniform01(n, dtype=np.float32, rng=None):
    rng = rng or rng_for("plain")
    return canonical(rng.random(n, dtype=np.float64).astype(dtype) if dtype != np.float32
                     else rng.random(n, dtype=np.float32))


def random_walk(n, dtype=np.float32, rng=None, chunk=1 << 24):
    """Cumulative sum of N(0,1) steps, accumulated in float64, then cast."""
    rng = rng or rng_for("large", 0)
    out = np.empty(n, dtype)
    acc = 0.0
    for s in range(0, n, chunk):
        e = min(n, s + chunk)
        steps = rng.standard_normal(e - s)
        np.cumsum(steps, out=steps)
        steps += acc
        acc = float(steps[-1])
        out[s:e] = steps.astype(dtype) if dtype != np.float64 else steps
    return canonical(out)


def piecewise_monotone(n, dtype=np.float32, rng=None, mean_run=100.0):
    """Alternating increasing / decreasing runs; run lengths geometric with the
    given mean, step sizes exponential(1); accumulated in float64."""
    rng = rng or rng_for("large", 1)
    runs = []
    total = 0
    while total < n:
        k = rng.geometric(1.0 / mean_run, size=max(16, int(2 * (n - total) / mean_run) + 16))
        runs.append(k)
        total += int(k.sum())
    runs = np.concatenate(runs)
    sign = np.where(np.arange(runs.size) % 2 == 0, 1.0, -1.0)
    signs = np.repeat(sign, runs)[:n]
    steps = rng.exponential(1.0, n) * signs
    np.cumsum(steps, out=steps)
    return canonical(steps.astype(dtype) if dtype != np.float64 else steps)


def ramp_f32(n):
    """Strictly increasing float32 series: consecutive bit patterns from 1.0
    (float(i) stops being strictly increasing past 2**24)."""
    if n > 0x7F7FFFFF - 0x3F800000:
        raise ValueError("ramp too long for float32")
    return (np.uint32(0x3F800000) + np.arange(n, dtype=np.uint32)).view(np.float32)


def uniform_i32(n, rng=None):
    rng = rng or rng_for("large", 3)
    return rng.integers(-2**31, 2**31, n, dtype=np.int64).astype(np.int32)


def uniform_u16(shape, rng=None):
    rng = rng or rng_for("image", 1)
    return rng.integers(0, 65536, shape, dtype=np.int64).astype(np.uint16)


def sine(n, period=10000.0, dtype=np.float64):
    """Sine wave of the given period (the paper's piecewise-monotone input)."""
    x = np.sin(2.0 * np.pi * np.arange(n, dtype=np.float64) / period)
    return canonical(x.astype(dtype))


def small_alphabet(n, k, dtype, rng):
    """Tie-heavy values: integers in [0, k) cast to dtype."""
    return rng.integers(0, k, n).astype(dtype)


def large_series(kind, n=1 << 28, dtype=np.float32):
    """The n = 2**28 single-series inputs: kind in {'walk', 'pwm', 'ramp', 'i32'}."""
    if kind == "walk":
        return random_walk(n, dtype, rng_for("large", 0))
    if kind == "pwm":
        return piecewise_monotone(n, dtype, rng_for("large", 1))
    if kind == "ramp":
        return ramp_f32(n)
    if kind == "i32":
        return uniform_i32(n, rng_for("large", 3))
    raise ValueError(kind)


# ------------------------------------------------------------------- images
def gaussian_field(rows, cols, sigma=16.0, noise=0.25, rng=None):
    """Smooth Gaussian random field (periodic Gaussian blur of white noise,
    normalised to unit std) plus noise * U[0,1), as float32."""
    rng = rng or rng_for("image", 0)
    white = rng.standard_normal((rows, cols)).astype(np.float32)
    fy = np.fft.fftfreq(rows).astype(np.float32)
    fx = np.fft.rfftfreq(cols).astype(np.float32)
    g = np.exp(-2.0 * (np.pi * sigma) ** 2 * (fy[:, None] ** 2 + fx[None, :] ** 2)).astype(np.float32)
    f = np.fft.rfft2(white)
    f *= g
    field = np.fft.irfft2(f, s=(rows, cols)).astype(np.float32)
    field /= np.float32(field.std() or 1.0)
    field += np.float32(noise) * rng.random((rows, cols), dtype=np.float32)
    return canonical(np.ascontiguousarray(field, np.float32))


# ---------------------------------------------------------------- batched
def batched_series(S=10000, lo=1000, hi=1000000, wlo=2, whi=1024, dtype=np.float32, rng=None):
    """Packed independent random walks.

    Returns ``(packed, in_offsets[S+1] int64, windows[S] int64)``.
    """
    rng = rng or rng_for("batched", 0)
    lens = np.floor(np.exp(rng.uniform(np.log(lo), np.log(hi), S))).astype(np.int64)
    wins = rng.integers(wlo, whi + 1, S).astype(np.int64)
    offs = np.zeros(S + 1, np.int64)
    np.cumsum(lens, out=offs[1:])
    packed = np.empty(int(offs[-1]), dtype)
    # one long walk, re-based at each series start: independent walks
    steps_rng = rng_for("batched", 1)
    chunk = 1 << 24
    for s in range(0, packed.size, chunk):
        e = min(packed.size, s + chunk)
        packed[s:e] = steps_rng.standard_normal(e - s).astype(dtype)
    for k in range(S):
        seg = packed[offs[k]:offs[k + 1]]
        np.cumsum(seg, out=seg, dtype=np.float64 if dtype == np.float64 else None)
    return canonical(packed), offs, wins


# ---------------------------------------------------------------- serving
def serving_requests(rate, duration, rng=None, n_lo=256, n_hi=4 << 20, w_lo=2, w_hi=8192,
                     dtypes=(np.float32, np.float64, np.int32)):
    """Open-loop Poisson filter requests: list of (arrival_s, dtype, n, w).

    Lengths are log-uniform in [n_lo, n_hi], windows uniform in [w_lo, w_hi];
    the dtype is uniform over ``dtypes``.
    """
    rng = rng or rng_for("serving", 0)
    t = 0.0
    out = []
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= duration:
            break
        dt = dtypes[int(rng.integers(0, len(dtypes)))]
        n = int(np.floor(np.exp(rng.uniform(np.log(n_lo), np.log(n_hi)))))
        w = int(rng.integers(w_lo, w_hi + 1))
        out.append((t, np.dtype(dt), n, w))
    return out


def stream_arrivals(n_streams, rate_per_stream, duration, rng=None):
    """Poisson chunk arrivals for persistent streams: sorted (time_s, stream_id)."""
    rng = rng or rng_for("serving", 1)
    ev = []
    for s in range(n_streams):
        t = rng.exponential(1.0 / rate_per_stream)
        while t < duration:
            ev.append((t, s))
            t += rng.exponential(1.0 / rate_per_stream)
    ev.sort()
    return ev


def request_payload(dtype, n, seed):
    """Series for one request: a random walk (floats) or uniform int32."""
    rng = np.random.default_rng(np.random.SeedSequence([SEED_ROOT, WORKLOAD_IDS["serving"], 1000003, int(seed)]))
    dtype = np.dtype(dtype)
    if dtype == np.int32:
        return uniform_i32(n, rng)
    return random_walk(n, dtype, rng)


# ------------------------------------------------------------ edge values
def _edge_specials(dtype):
    dtype = np.dtype(dtype)
    if dtype.kind == "f":
        fi = np.finfo(dtype)
        ub = {4: np.uint32, 8: np.uint64}[dtype.itemsize]
        sub_min = np.array([1], ub).view(dtype)[0]
        sub_max = np.array([(1 << fi.nmant) - 1], ub).view(dtype)[0]
        v = [-np.inf, np.inf, -0.0, sub_min, -sub_min, sub_max, -sub_max, fi.tiny, -fi.tiny,
             fi.max, -fi.max, 1.0, -1.0]
        return np.array(v, dtype)
    if dtype == np.int32:
        return np.array([-2**31, -2**31 + 1, -1, 0, 1, 2**31 - 2, 2**31 - 1], np.int32)
    if dtype == np.uint16:
        return np.array([0, 1, 32767, 32768, 65534, 65535], np.uint16)
    raise ValueError(dtype)


def _random_bits(n, dtype, rng):
    """Values drawn uniformly over the type's bit patterns: for floats every
    NaN pattern becomes -inf and +0.0 becomes -0.0 (so a window never holds
    both zeros, whose selected bits the contract leaves unspecified)."""
    dtype = np.dtype(dtype)
    if dtype.kind != "f":
        info = np.iinfo(dtype)
        return rng.integers(int(info.min), int(info.max) + 1, n, dtype=np.int64).astype(dtype)
    ub = {4: np.uint32, 8: np.uint64}[dtype.itemsize]
    bitsv = rng.integers(0, np.iinfo(ub).max, n, dtype=ub, endpoint=True)
    x = bitsv.view(dtype)
    x[np.isnan(x)] = -np.inf
    x[x == 0] = -0.0
    return x


def edge_series(n, dtype, rng, special_frac=0.4):
    """Series made of the values a selection kernel is most likely to get
    wrong: +-inf, -0.0 (never +0.0), subnormals, the largest finite and
    smallest normal values, integer extremes (INT32_MIN/MAX, uint16 0 and
    65535, i.e. the identities of the running max and min), and values
    uniform over the type's bit patterns.  Values come in runs: mostly
    short, some of ~100 and a few of 1000-20000 samples, so whole windows
    hold a single extreme value.  NaN-free."""
    dtype = np.dtype(dtype)
    if n == 0:
        return np.zeros(0, dtype)
    runs = []
    total = 0
    while total < n:
        u = rng.random()
        k = int(rng.geometric(1 / 3.0)) if u < 0.7 else (int(rng.geometric(1 / 100.0)) if u < 0.95
                                                          else int(rng.integers(1000, 20001)))
        runs.append(k)
        total += k
    runs = np.array(runs, np.int64)
    spec = _edge_specials(dtype)
    pick = rng.random(runs.size) < special_frac
    vals = _random_bits(runs.size, dtype, rng)
    vals[pick] = spec[rng.integers(0, spec.size, int(pick.sum()))]
    return np.repeat(vals, runs)[:n].copy()
