"""MI355X-native (gfx950) running max-min filter.

The compute path is libmaxmin.so: hand-written HIP kernels behind the C ABI in
``include/maxmin.h``.  This package holds its build script (``build``), the thin
ctypes binding (``binding``; same names as the C entry points) and the seeded
synthetic input generators (``synth``).  Importing the package loads nothing;
the binding loads the library on first use and raises if it is missing.
"""
__all__ = ["maxmin_filter", "maxmin_filter_batched", "maxmin_out_offsets", "maxmin_stream_create",
           "MaxMinStream", "maxmin_filter_2d", "maxmin_set_strategy", "maxmin_plan", "maxmin_check_stream",
           "maxmin_last_error", "maxmin_version", "MaxMinError", "MaxMinEngine"]


def __getattr__(name):
    if name in __all__:
        from . import binding
        return getattr(binding, name)
    raise AttributeError(name)
