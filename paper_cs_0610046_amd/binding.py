"""Thin Python binding of libmaxmin's C ABI (``include/maxmin.h``).

Argument marshalling only: every step of the filter runs in the library's
gfx950 kernels.  Functions carry the C names; array arguments are torch CUDA
tensors (device memory and streams are torch's), offsets for the host helper
are numpy arrays.  If the library has not been built, every entry point
raises -- there is no fallback.
"""
import ctypes
import os
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_build", "libmaxmin.so")

MAXMIN_OK, MAXMIN_EINVAL, MAXMIN_ENOMEM, MAXMIN_EDEVICE, MAXMIN_EBUSY, MAXMIN_EUNSUPPORTED = 0, -1, -2, -3, -4, -5
STRATEGY_AUTO, STRATEGY_TILE, STRATEGY_CHUNK, STRATEGY_RUN = 0, 1, 2, 3

_lock = threading.Lock()
_lib = None


class MaxMinError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("maxmin error %d: %s" % (code, msg))
        self.code = code


def lib():
    """Load libmaxmin.so (built by ``paper_cs_0610046_amd.build``)."""
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libmaxmin.so is not built (%s); run __graft_entry__.build() or "
                               "python paper_cs_0610046_amd/build.py" % LIB_PATH)
        L = ctypes.CDLL(LIB_PATH)
        i64, vp, ci = ctypes.c_int64, ctypes.c_void_p, ctypes.c_int
        i64p = ctypes.POINTER(ctypes.c_int64)
        L.maxmin_filter.argtypes = [ci, vp, i64, i64, vp, vp, vp]
        L.maxmin_filter_noalloc.argtypes = [ci, vp, i64, i64, vp, vp, vp]
        L.maxmin_argfilter.argtypes = [ci, vp, i64, i64, vp, vp, vp, vp, vp]
        L.maxmin_filter_batched.argtypes = [ci, vp, vp, vp, vp, i64, vp, vp, vp]
        L.maxmin_out_offsets.argtypes = [vp, vp, i64, vp]
        L.maxmin_stream_create.argtypes = [ci, i64, ctypes.POINTER(vp)]
        L.maxmin_stream_push.argtypes = [vp, vp, i64, vp, vp, i64p, vp]
        L.maxmin_stream_destroy.argtypes = [vp]
        L.maxmin_stream_samples.argtypes = [vp]
        L.maxmin_stream_samples.restype = i64
        L.maxmin_stream_export.argtypes = [vp, vp, i64p]
        L.maxmin_stream_import.argtypes = [ci, i64, i64, vp, ctypes.POINTER(vp)]
        L.maxmin_filter_2d.argtypes = [ci, vp, i64, i64, i64, i64, i64, vp, vp, i64, vp]
        L.maxmin_morph_2d.argtypes = [ci, vp, i64, i64, i64, i64, i64, ci, vp, i64, vp]
        L.maxmin_autotune.argtypes = [ci, i64, vp]
        L.maxmin_tuning.argtypes = [ci, i64p]
        L.maxmin_envelope.argtypes = [ci, vp, i64, i64, vp, vp, vp]
        L.maxmin_envelope_batched.argtypes = [ci, vp, vp, vp, i64, vp, vp, vp]
        L.maxmin_set_strategy.argtypes = [ci]
        L.maxmin_plan.argtypes = [ci, i64, i64]
        L.maxmin_plan_2d.argtypes = [ci, i64, i64, ci]
        L.maxmin_check_stream.argtypes = [vp]
        vpp = ctypes.POINTER(vp)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        L.maxmin_engine_create.argtypes = [i64, ci, i64, vpp]
        L.maxmin_engine_open_stream.argtypes = [vp, ci, i64, i64p]
        L.maxmin_engine_close_stream.argtypes = [vp, i64]
        L.maxmin_engine_submit_filter.argtypes = [vp, ci, vp, i64, i64, vp, vp, i64p]
        L.maxmin_engine_submit_push.argtypes = [vp, i64, vp, i64, vp, vp, i64p]
        L.maxmin_engine_poll.argtypes = [vp, i64p, i64p, dp, ip, i64, i64p]
        L.maxmin_engine_drain.argtypes = [vp]
        L.maxmin_engine_stats.argtypes = [vp, i64p]
        L.maxmin_engine_replay.argtypes = [vp, i64, dp, ip, ip, i64p, i64p, i64p, vpp, vpp, vpp, i64p, dp]
        L.maxmin_engine_destroy.argtypes = [vp]
        for f in ("maxmin_engine_create", "maxmin_engine_open_stream", "maxmin_engine_close_stream",
                  "maxmin_engine_submit_filter", "maxmin_engine_submit_push", "maxmin_engine_poll",
                  "maxmin_engine_drain", "maxmin_engine_stats", "maxmin_engine_replay", "maxmin_engine_destroy"):
            getattr(L, f).restype = ci
        L.maxmin_last_error.restype = ctypes.c_char_p
        L.maxmin_version.restype = ctypes.c_char_p
        for f in ("maxmin_filter", "maxmin_filter_noalloc", "maxmin_argfilter", "maxmin_filter_batched", "maxmin_out_offsets", "maxmin_stream_create",
                  "maxmin_stream_push", "maxmin_stream_destroy", "maxmin_stream_export", "maxmin_stream_import", "maxmin_filter_2d", "maxmin_morph_2d",
                  "maxmin_envelope", "maxmin_envelope_batched", "maxmin_autotune", "maxmin_tuning",
                  "maxmin_set_strategy",
                  "maxmin_plan", "maxmin_plan_2d", "maxmin_check_stream"):
            getattr(L, f).restype = ci
        _lib = L
        return L


def _check(code):
    if code != MAXMIN_OK:
        raise MaxMinError(code, lib().maxmin_last_error().decode())


_TORCH_CODES = None


def dtype_code(dtype):
    """maxmin_dtype_t of a torch or numpy dtype."""
    global _TORCH_CODES
    if _TORCH_CODES is None:
        import torch
        _TORCH_CODES = {torch.float32: 0, torch.float64: 1, torch.int32: 2, torch.uint16: 3}
    if dtype in _TORCH_CODES:
        return _TORCH_CODES[dtype]
    d = np.dtype(dtype)
    return {np.dtype(np.float32): 0, np.dtype(np.float64): 1, np.dtype(np.int32): 2, np.dtype(np.uint16): 3}[d]


def _np_dtype(dtype):
    """The numpy dtype of a torch or numpy dtype."""
    return [np.float32, np.float64, np.int32, np.uint16][dtype_code(dtype)]


def _stream(stream):
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None and t.numel() else ctypes.c_void_p(0)


def _cuda_1d(t, name):
    if not t.is_cuda:
        raise ValueError("%s must be a CUDA (HIP) tensor" % name)
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    return t


def n_out(n, w):
    return max(0, int(n) - int(w) + 1)


def _want(which):
    if which not in ("both", "max", "min"):
        raise ValueError("which must be 'both', 'max' or 'min'")
    return which != "min", which != "max"


def maxmin_filter(x, w, out_max=None, out_min=None, stream=None, which="both"):
    """Running max and min of every window [j, j+w) of the 1-D tensor x.
    ``which="max"`` / ``"min"``: a max-only / min-only filter (the other
    output is None and is not computed into memory)."""
    import torch
    _cuda_1d(x, "x")
    k = n_out(x.numel(), w)
    wx, wn = _want(which)
    if out_max is None and wx:
        out_max = torch.empty(k, dtype=x.dtype, device=x.device)
    if out_min is None and wn:
        out_min = torch.empty(k, dtype=x.dtype, device=x.device)
    out_max, out_min = (out_max if wx else None), (out_min if wn else None)
    _check(lib().maxmin_filter(dtype_code(x.dtype), _ptr(x), x.numel(), int(w), _ptr(out_max), _ptr(out_min),
                               _stream(stream)))
    return out_max, out_min


def maxmin_filter_noalloc(x, w, out_max, out_min, stream=None):
    """maxmin_filter into caller-given outputs with no allocation by the
    library (its long-window scratch is a fixed device array)."""
    _cuda_1d(x, "x")
    _check(lib().maxmin_filter_noalloc(dtype_code(x.dtype), _ptr(x), x.numel(), int(w), _ptr(out_max),
                                       _ptr(out_min), _stream(stream)))
    return out_max, out_min


def maxmin_argfilter(x, w, out_max=None, out_min=None, out_argmax=None, out_argmin=None, stream=None):
    """Window max and min of the 1-D tensor x with the leftmost location of
    each (int64 positions in x).  Returns (max, min, argmax, argmin)."""
    import torch
    _cuda_1d(x, "x")
    k = n_out(x.numel(), w)
    out_max = torch.empty(k, dtype=x.dtype, device=x.device) if out_max is None else out_max
    out_min = torch.empty(k, dtype=x.dtype, device=x.device) if out_min is None else out_min
    out_argmax = torch.empty(k, dtype=torch.int64, device=x.device) if out_argmax is None else out_argmax
    out_argmin = torch.empty(k, dtype=torch.int64, device=x.device) if out_argmin is None else out_argmin
    _check(lib().maxmin_argfilter(dtype_code(x.dtype), _ptr(x), x.numel(), int(w), _ptr(out_max), _ptr(out_min),
                                  _ptr(out_argmax), _ptr(out_argmin), _stream(stream)))
    return out_max, out_min, out_argmax, out_argmin


def maxmin_out_offsets(in_offsets, windows):
    """Host helper: output offsets of a packed batch (numpy int64 arrays)."""
    in_offsets = np.ascontiguousarray(in_offsets, np.int64)
    windows = np.ascontiguousarray(windows, np.int64)
    S = windows.size
    out = np.zeros(S + 1, np.int64)
    _check(lib().maxmin_out_offsets(in_offsets.ctypes.data, windows.ctypes.data if S else None, S,
                                    out.ctypes.data))
    return out


def maxmin_filter_batched(packed, in_offsets, windows, out_offsets, out_max=None, out_min=None, stream=None,
                          which="both"):
    """S series packed in one tensor, each with its own window.

    ``in_offsets`` (S+1), ``windows`` (S) and ``out_offsets`` (S+1) are int64
    CUDA tensors; ``out_offsets`` comes from :func:`maxmin_out_offsets`.
    ``total_out`` outputs are allocated if not given (needs out_offsets[-1]
    on the host: pass the outputs to avoid that read).
    """
    import torch
    _cuda_1d(packed, "packed")
    S = windows.numel()
    wx, wn = _want(which)
    if (out_max is None and wx) or (out_min is None and wn):
        total = int(out_offsets[-1].item()) if S else 0
        out_max = torch.empty(total, dtype=packed.dtype, device=packed.device) if out_max is None else out_max
        out_min = torch.empty(total, dtype=packed.dtype, device=packed.device) if out_min is None else out_min
    out_max, out_min = (out_max if wx else None), (out_min if wn else None)
    _check(lib().maxmin_filter_batched(dtype_code(packed.dtype), _ptr(packed), _ptr(in_offsets), _ptr(windows),
                                       _ptr(out_offsets), S, _ptr(out_max), _ptr(out_min), _stream(stream)))
    return out_max, out_min


class MaxMinStream:
    """maxmin_stream_create / push / destroy: zero-latency chunked filtering;
    export / import of the stream's state (t, last min(t, w-1) samples)."""

    def __init__(self, dtype, w, _handle=None):
        self.dtype = dtype
        self.w = int(w)
        if _handle is not None:
            self._h = _handle
            return
        h = ctypes.c_void_p()
        _check(lib().maxmin_stream_create(dtype_code(dtype), self.w, ctypes.byref(h)))
        self._h = h

    def export(self):
        """(t, carry): carry a host numpy array of the last min(t, w-1) samples."""
        t = ctypes.c_int64(0)
        c = max(0, min(self.samples, self.w - 1))
        carry = np.empty(c, dtype=_np_dtype(self.dtype))
        _check(lib().maxmin_stream_export(self._h, carry.ctypes.data if c else None, ctypes.byref(t)))
        return t.value, carry

    def push(self, chunk, out_max=None, out_min=None, stream=None, which="both"):
        import torch
        _cuda_1d(chunk, "chunk")
        m = chunk.numel()
        wx, wn = _want(which)
        if out_max is None and wx:
            out_max = torch.empty(m, dtype=chunk.dtype, device=chunk.device)
        if out_min is None and wn:
            out_min = torch.empty(m, dtype=chunk.dtype, device=chunk.device)
        out_max, out_min = (out_max if wx else None), (out_min if wn else None)
        k = ctypes.c_int64(0)
        _check(lib().maxmin_stream_push(self._h, _ptr(chunk), m, _ptr(out_max), _ptr(out_min), ctypes.byref(k),
                                        _stream(stream)))
        return (out_max[:k.value] if wx else None), (out_min[:k.value] if wn else None)

    @property
    def samples(self):
        return lib().maxmin_stream_samples(self._h)

    def close(self):
        if self._h:
            lib().maxmin_stream_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def maxmin_stream_create(dtype, w):
    return MaxMinStream(dtype, w)


def maxmin_stream_import(dtype, w, t, carry):
    """A stream that continues from an exported state (t, carry)."""
    carry = np.ascontiguousarray(carry, dtype=_np_dtype(dtype))
    if carry.size != max(0, min(int(t), int(w) - 1)):
        raise ValueError("carry must hold min(t, w-1) samples")
    h = ctypes.c_void_p()
    _check(lib().maxmin_stream_import(dtype_code(dtype), int(w), int(t), carry.ctypes.data if carry.size else None,
                                      ctypes.byref(h)))
    return MaxMinStream(dtype, w, _handle=h)


def _check_img(img):
    if not img.is_cuda or img.dim() != 2 or img.stride(1) != 1:
        raise ValueError("img must be a 2-D CUDA tensor with unit column stride")


def maxmin_filter_2d(img, w_rows, w_cols=None, out_max=None, out_min=None, stream=None, which="both"):
    """Rows, then columns: max/min over every w_rows x w_cols rectangle."""
    import torch
    _check_img(img)
    w_cols = w_rows if w_cols is None else w_cols
    rows, cols = img.shape
    orr, occ = n_out(rows, w_rows), n_out(cols, w_cols)
    wx, wn = _want(which)
    if out_max is None and wx:
        out_max = torch.empty((orr, occ), dtype=img.dtype, device=img.device)
    if out_min is None and wn:
        out_min = torch.empty((orr, occ), dtype=img.dtype, device=img.device)
    out_max, out_min = (out_max if wx else None), (out_min if wn else None)
    if out_max is not None and out_min is not None and orr and occ and out_max.stride(0) != out_min.stride(0):
        raise ValueError("out_max and out_min must share one leading dimension")
    ref = out_max if out_max is not None else out_min
    ld_out = ref.stride(0) if orr and occ else max(occ, 1)
    _check(lib().maxmin_filter_2d(dtype_code(img.dtype), _ptr(img), rows, cols, img.stride(0) if rows else cols,
                                  int(w_rows), int(w_cols), _ptr(out_max), _ptr(out_min), ld_out, _stream(stream)))
    return out_max, out_min


def maxmin_envelope(x, r, out_upper=None, out_lower=None, stream=None):
    """Centered envelope of radius r: max / min over [i-r, i+r] truncated at
    the ends (n outputs each).  Returns (upper, lower)."""
    import torch
    _cuda_1d(x, "x")
    out_upper = torch.empty_like(x) if out_upper is None else out_upper
    out_lower = torch.empty_like(x) if out_lower is None else out_lower
    _check(lib().maxmin_envelope(dtype_code(x.dtype), _ptr(x), x.numel(), int(r), _ptr(out_upper), _ptr(out_lower),
                                 _stream(stream)))
    return out_upper, out_lower


def maxmin_envelope_batched(packed, in_offsets, radii, out_upper=None, out_lower=None, stream=None):
    """Envelopes of S packed series (device int64 ``in_offsets`` [S+1] and
    ``radii`` [S]), packed like the input."""
    import torch
    _cuda_1d(packed, "packed")
    out_upper = torch.empty_like(packed) if out_upper is None else out_upper
    out_lower = torch.empty_like(packed) if out_lower is None else out_lower
    _check(lib().maxmin_envelope_batched(dtype_code(packed.dtype), _ptr(packed), _ptr(in_offsets), _ptr(radii),
                                         radii.numel(), _ptr(out_upper), _ptr(out_lower), _stream(stream)))
    return out_upper, out_lower


def maxmin_autotune(dtype, n=0, stream=None):
    """Measure the planner's launch parameters for ``dtype`` on this device
    (process-wide) and return the resulting table (see :func:`maxmin_tuning`)."""
    _check(lib().maxmin_autotune(dtype_code(dtype), int(n), _stream(stream)))
    return maxmin_tuning(dtype)


TUNING_LEN = 17
BATCH_WCLASSES = ("w<=2048", "w<=4096", "w<=8192")
BATCH_NCLASSES = ("n<2^16", "n<2^20", "n>=2^20")


def maxmin_tuning(dtype):
    """The planner's launch parameters for ``dtype`` (host only): run
    lengths, ticket ranges, the long-window strategy and the batched plan
    (tile size and, per size class, "tile" or "chunk")."""
    out = (ctypes.c_int64 * TUNING_LEN)()
    _check(lib().maxmin_tuning(dtype_code(dtype), out))
    plan = {}
    for wc, wn in enumerate(BATCH_WCLASSES):
        for nc, nn in enumerate(BATCH_NCLASSES):
            plan["%s,%s" % (wn, nn)] = "tile" if out[7 + 3 * wc + nc] == 0 else "chunk"
    return {"tile_run_subtiles": out[0], "tile_run_subtiles_long": out[1], "rows_run_subtiles": out[2],
            "chunk_ranges_one_chunk": out[3], "chunk_ranges_long": out[4],
            "long_window_strategy": {2: "chunk", 3: "run"}.get(out[5], out[5]),
            "batched_tile_subtiles": out[6], "batched_plan": plan, "measured": bool(out[16])}


MORPH_OPS = {"erode": 0, "dilate": 1, "open": 2, "close": 3}


def maxmin_morph_2d(img, op, w_rows, w_cols=None, out=None, stream=None):
    """Grey-scale erosion / dilation / opening / closing with a w_rows x
    w_cols rectangle (valid windows; opening and closing shrink twice)."""
    import torch
    _check_img(img)
    w_cols = w_rows if w_cols is None else w_cols
    code = MORPH_OPS[op] if isinstance(op, str) else int(op)
    rows, cols = img.shape
    k = 1 if code < 2 else 2
    orr = max(0, rows - k * (int(w_rows) - 1))
    occ = max(0, cols - k * (int(w_cols) - 1))
    if out is None:
        out = torch.empty((orr, occ), dtype=img.dtype, device=img.device)
    ld_out = out.stride(0) if orr and occ else max(occ, 1)
    _check(lib().maxmin_morph_2d(dtype_code(img.dtype), _ptr(img), rows, cols, img.stride(0) if rows else cols,
                                 int(w_rows), int(w_cols), code, _ptr(out), ld_out, _stream(stream)))
    return out


def maxmin_set_strategy(strategy):
    _check(lib().maxmin_set_strategy(int(strategy)))


def maxmin_plan(dtype, n, w):
    return lib().maxmin_plan(dtype_code(dtype), int(n), int(w))


PLAN_2D_FUSED, PLAN_2D_ROWS_COLS = 1, 2


def maxmin_plan_2d(dtype, w_rows, w_cols, outputs=2):
    """PLAN_2D_FUSED (one pass) or PLAN_2D_ROWS_COLS for these windows, for
    a call with both outputs (outputs=2) or one (outputs=1)."""
    r = lib().maxmin_plan_2d(dtype_code(dtype), int(w_rows), int(w_cols), int(outputs))
    if r not in (PLAN_2D_FUSED, PLAN_2D_ROWS_COLS):
        _check(r)
    return r


def maxmin_check_stream(stream=None):
    _check(lib().maxmin_check_stream(_stream(stream)))


def maxmin_last_error():
    return lib().maxmin_last_error().decode()


def maxmin_version():
    return lib().maxmin_version().decode()


def _hptr(a):
    """Host address of a numpy array or a CPU torch tensor."""
    if a is None:
        return ctypes.c_void_p(0)
    if hasattr(a, "data_ptr"):
        return ctypes.c_void_p(a.data_ptr())
    return ctypes.c_void_p(a.ctypes.data)


class MaxMinEngine:
    """maxmin_engine_*: serving loop with HBM admission and continuous
    batching.  Buffers are host arrays (numpy, or pinned CPU torch tensors);
    they must stay alive until their request is polled."""

    def __init__(self, budget_bytes=64 << 30, lanes=4, max_batch=256):
        h = ctypes.c_void_p()
        _check(lib().maxmin_engine_create(int(budget_bytes), int(lanes), int(max_batch), ctypes.byref(h)))
        self._h = h
        self._keep = {}

    def open_stream(self, dtype, w):
        sid = ctypes.c_int64()
        _check(lib().maxmin_engine_open_stream(self._h, dtype_code(dtype), int(w), ctypes.byref(sid)))
        return sid.value

    def close_stream(self, sid):
        _check(lib().maxmin_engine_close_stream(self._h, int(sid)))

    def submit_filter(self, h_in, w, h_max, h_min, dtype=None):
        rid = ctypes.c_int64()
        dt = dtype_code(dtype if dtype is not None else h_in.dtype)
        n = h_in.numel() if hasattr(h_in, "numel") else h_in.size
        _check(lib().maxmin_engine_submit_filter(self._h, dt, _hptr(h_in), n, int(w), _hptr(h_max), _hptr(h_min),
                                                 ctypes.byref(rid)))
        self._keep[rid.value] = (h_in, h_max, h_min)
        return rid.value

    def submit_push(self, sid, h_chunk, h_max, h_min):
        rid = ctypes.c_int64()
        m = h_chunk.numel() if hasattr(h_chunk, "numel") else h_chunk.size
        _check(lib().maxmin_engine_submit_push(self._h, int(sid), _hptr(h_chunk), m, _hptr(h_max), _hptr(h_min),
                                               ctypes.byref(rid)))
        self._keep[rid.value] = (h_chunk, h_max, h_min)
        return rid.value

    def poll(self, cap=65536):
        """Finished requests: list of (id, n_out, latency_s, status)."""
        ids = (ctypes.c_int64 * cap)()
        no = (ctypes.c_int64 * cap)()
        lat = (ctypes.c_double * cap)()
        st = (ctypes.c_int * cap)()
        got = ctypes.c_int64()
        _check(lib().maxmin_engine_poll(self._h, ids, no, lat, st, cap, ctypes.byref(got)))
        out = [(ids[i], no[i], lat[i], st[i]) for i in range(got.value)]
        for r in out:
            self._keep.pop(r[0], None)
        return out

    def drain(self):
        _check(lib().maxmin_engine_drain(self._h))

    def stats(self):
        a = (ctypes.c_int64 * 9)()
        _check(lib().maxmin_engine_stats(self._h, a))
        keys = ("submitted", "finished", "batches", "rejected", "samples", "bytes_in_use", "peak_bytes", "pending",
                "refused")
        return dict(zip(keys, list(a)))

    def replay(self, at_s, kind, dtype, n, w, sid, h_in, h_max, h_min):
        """Open-loop submission from a C++ thread (blocks until the last
        request is submitted).  Returns (request ids, submission lag)."""
        cnt = len(at_s)
        A = lambda t, v: (t * cnt)(*v)  # noqa: E731
        ids = (ctypes.c_int64 * cnt)()
        lag = (ctypes.c_double * cnt)()
        _check(lib().maxmin_engine_replay(
            self._h, cnt, A(ctypes.c_double, at_s), A(ctypes.c_int, kind), A(ctypes.c_int, dtype),
            A(ctypes.c_int64, n), A(ctypes.c_int64, w), A(ctypes.c_int64, sid),
            A(ctypes.c_void_p, h_in), A(ctypes.c_void_p, h_max), A(ctypes.c_void_p, h_min), ids, lag))
        return list(ids), list(lag)

    def close(self):
        if self._h:
            _check(lib().maxmin_engine_destroy(self._h))
            self._h = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
