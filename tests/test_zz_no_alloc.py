"""maxmin_filter_noalloc (no allocation; scratch in a fixed device array)
against maxmin_filter through the C ABI, bit-exact: two calls in a row per
window class, the second on a smaller input (the array keeps the first
call's contents), every dtype; sizes beyond the array are refused."""
import ctypes

import numpy as np
import pytest

from paper_cs_0610046_amd import binding as mm
from paper_cs_0610046_amd import synth
from gpu_util import assert_bits_equal, note, to_dev, to_host

pytestmark = pytest.mark.gpu


def _noalloc(x, w):
    import torch
    L = mm.lib()
    f = L.maxmin_filter_noalloc
    f.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                  ctypes.c_void_p]
    f.restype = ctypes.c_int
    k = max(0, x.numel() - w + 1)
    mx = torch.empty(k, dtype=x.dtype, device=x.device)
    mn = torch.empty(k, dtype=x.dtype, device=x.device)
    rc = f(mm.dtype_code(x.dtype), ctypes.c_void_p(x.data_ptr()), x.numel(), w,
           ctypes.c_void_p(mx.data_ptr() if k else 0), ctypes.c_void_p(mn.data_ptr() if k else 0),
           ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == 0, mm.maxmin_last_error()
    return mx, mn


@pytest.mark.parametrize("dt", [np.float32, np.float64, np.int32, np.uint16], ids=lambda d: np.dtype(d).name)
def test_noalloc_equals_filter(dt):
    import torch
    rng = synth.rng_for("tests", 950)
    first = synth.random_walk((1 << 22) + 17, np.float64, rng)
    second = synth.random_walk(300007, np.float64, rng)
    cast = (lambda a: a.astype(dt)) if dt in (np.float32, np.float64) else \
        (lambda a: (np.round(a * 100).astype(np.int64) % 60000).astype(dt))
    for w in (1, 300, 3000, 5000, 8192, 9000, 40000, 65536, 100000, 299999):
        for a in (cast(first), cast(second)):
            x = to_dev(a)
            note("noalloc dt=%s n=%d w=%d" % (np.dtype(dt).name, a.size, w))
            gx, gn = _noalloc(x, w)
            fx, fn = mm.maxmin_filter(x, w)
            torch.cuda.synchronize()
            assert_bits_equal(to_host(gx, dt), to_host(fx, dt), "noalloc max n=%d w=%d" % (a.size, w))
            assert_bits_equal(to_host(gn, dt), to_host(fn, dt), "noalloc min n=%d w=%d" % (a.size, w))


def test_noalloc_refuses_beyond_scratch():
    """A long-window series whose chunk aggregates exceed the 32 MiB array is
    refused before anything is launched (the pointers are never touched)."""
    L = mm.lib()
    f = L.maxmin_filter_noalloc
    f.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                  ctypes.c_void_p]
    f.restype = ctypes.c_int
    vp = ctypes.c_void_p
    assert f(1, vp(0x1000), 1 << 34, 10000, vp(0x2000), vp(0x3000), None) == mm.MAXMIN_EUNSUPPORTED
