"""Host-side checks of the C ABI (no GPU): the library loads, exports every
entry point declared in include/maxmin.h, and its host-only paths (argument
checks, the out-offsets helper, the planner) behave as documented."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
from paper_cs_0610046_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "maxmin.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(maxmin_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(binding.LIB_PATH):
        from paper_cs_0610046_amd import build
        build.build()
    return binding.lib()


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("maxmin_filter", "maxmin_argfilter", "maxmin_filter_batched", "maxmin_out_offsets", "maxmin_stream_create",
              "maxmin_stream_push", "maxmin_stream_destroy", "maxmin_filter_2d", "maxmin_last_error"):
        assert n in names


def test_every_declared_symbol_is_exported(lib):
    for n in declared_functions():
        assert hasattr(lib, n), n
        assert ctypes.cast(getattr(lib, n), ctypes.c_void_p).value


def test_argument_errors_without_gpu(lib):
    vp = ctypes.c_void_p
    assert lib.maxmin_filter(0, None, 10, 0, None, None, None) == binding.MAXMIN_EINVAL
    assert "w=0" in binding.maxmin_last_error()
    assert lib.maxmin_filter(7, None, 10, 2, None, None, None) == binding.MAXMIN_EINVAL
    assert lib.maxmin_filter(0, None, -1, 2, None, None, None) == binding.MAXMIN_EINVAL
    # w > n: no output, not an error, nothing touched
    assert lib.maxmin_filter(0, None, 10, 11, None, None, None) == binding.MAXMIN_OK
    assert lib.maxmin_filter(0, None, 0, 1, None, None, None) == binding.MAXMIN_OK
    # work to do but null pointers
    assert lib.maxmin_filter(0, None, 10, 3, None, None, None) == binding.MAXMIN_EINVAL
    # misaligned pointer (checked before any device call)
    assert lib.maxmin_filter(0, vp(0x1002), 10, 3, vp(0x2000), vp(0x3000), None) == binding.MAXMIN_EINVAL
    assert lib.maxmin_filter_batched(0, None, None, None, None, -1, None, None, None) == binding.MAXMIN_EINVAL
    assert lib.maxmin_filter_batched(0, None, None, None, None, 0, None, None, None) == binding.MAXMIN_OK
    assert lib.maxmin_filter_2d(0, None, 5, 5, 4, 2, 2, None, None, 4, None) == binding.MAXMIN_EINVAL  # ld < cols
    assert lib.maxmin_filter_2d(0, None, 5, 5, 5, 6, 2, None, None, 4, None) == binding.MAXMIN_OK  # no output
    assert lib.maxmin_argfilter(0, None, 10, 0, None, None, None, None, None) == binding.MAXMIN_EINVAL
    assert lib.maxmin_argfilter(0, None, 10, 11, None, None, None, None, None) == binding.MAXMIN_OK
    assert lib.maxmin_argfilter(0, vp(0x1000), 10, 3, vp(0x2000), vp(0x3000), None, vp(0x4000), None) == \
        binding.MAXMIN_EINVAL
    assert lib.maxmin_argfilter(0, vp(0x1000), 10, 3, vp(0x2000), vp(0x3000), vp(0x4004), vp(0x5000), None) == \
        binding.MAXMIN_EINVAL  # location output not 8-byte aligned
    # no-allocation entry point: argument checks, and a long window whose
    # aggregates exceed its fixed scratch is refused before any device call
    assert lib.maxmin_filter_noalloc(0, None, 10, 0, None, None, None) == binding.MAXMIN_EINVAL
    assert lib.maxmin_filter_noalloc(0, None, 10, 11, None, None, None) == binding.MAXMIN_OK
    assert lib.maxmin_filter_noalloc(0, vp(0x1002), 10, 3, vp(0x2000), vp(0x3000), None) == binding.MAXMIN_EINVAL
    assert lib.maxmin_filter_noalloc(1, vp(0x1000), 1 << 34, 10000, vp(0x2000), vp(0x3000), None) == \
        binding.MAXMIN_EUNSUPPORTED
    assert "32 MiB" in binding.maxmin_last_error()
    assert lib.maxmin_set_strategy(9) == binding.MAXMIN_EINVAL
    assert lib.maxmin_set_strategy(3) == binding.MAXMIN_OK
    assert lib.maxmin_set_strategy(0) == binding.MAXMIN_OK
    h = ctypes.c_void_p()
    assert lib.maxmin_stream_create(0, 0, ctypes.byref(h)) == binding.MAXMIN_EINVAL
    assert lib.maxmin_stream_push(None, None, 4, None, None, None, None) == binding.MAXMIN_EINVAL
    assert lib.maxmin_stream_destroy(None) == binding.MAXMIN_OK
    assert lib.maxmin_stream_samples(None) == -1
    t = ctypes.c_int64(0)
    assert lib.maxmin_stream_export(None, None, ctypes.byref(t)) == binding.MAXMIN_EINVAL
    assert lib.maxmin_stream_import(0, 8, -1, None, ctypes.byref(h)) == binding.MAXMIN_EINVAL
    assert lib.maxmin_stream_import(0, 0, 3, None, ctypes.byref(h)) == binding.MAXMIN_EINVAL
    assert lib.maxmin_stream_import(7, 8, 3, None, ctypes.byref(h)) == binding.MAXMIN_EINVAL
    assert lib.maxmin_stream_import(0, 8, 3, None, ctypes.byref(h)) == binding.MAXMIN_EINVAL  # 3 samples, no carry
    assert lib.maxmin_stream_import(0, 8, 3, None, None) == binding.MAXMIN_EINVAL


def test_tuning_table_and_autotune_arguments(lib):
    t = binding.maxmin_tuning(np.float32)
    plan = t.pop("batched_plan")
    assert t == {"tile_run_subtiles": 4, "tile_run_subtiles_long": 64, "rows_run_subtiles": 16,
                 "chunk_ranges_one_chunk": 16, "chunk_ranges_long": 0, "long_window_strategy": "chunk",
                 "batched_tile_subtiles": 1, "measured": False}
    assert len(plan) == 9 and set(plan.values()) == {"tile"}  # default: the tile kernel for every class
    assert lib.maxmin_autotune(9, 0, None) == binding.MAXMIN_EINVAL
    assert lib.maxmin_autotune(0, 1000, None) == binding.MAXMIN_EINVAL  # below 2^20, checked before any device call
    assert lib.maxmin_tuning(9, None) == binding.MAXMIN_EINVAL


def test_out_offsets_matches_oracle(lib):
    rng = np.random.default_rng(3)
    lens = rng.integers(0, 50, 200)
    offs = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    wins = rng.integers(1, 60, 200).astype(np.int64)
    assert np.array_equal(binding.maxmin_out_offsets(offs, wins), oracle.out_offsets(offs, wins))
    with pytest.raises(binding.MaxMinError):
        binding.maxmin_out_offsets(np.array([0, 5, 3], np.int64), np.array([1, 1], np.int64))
    with pytest.raises(binding.MaxMinError):
        binding.maxmin_out_offsets(np.array([0, 5], np.int64), np.array([0], np.int64))


def test_planner_2d(lib, monkeypatch):
    """The 2-D path choice: the fused pass for the windows it fits (w_rows
    <= 64, w_cols <= 64 V + 1) up to w_rows 15, or 23 for 16-bit data with
    both outputs; rows then columns beyond."""
    monkeypatch.delenv("MAXMIN_2D_FUSED", raising=False)
    F, RC = binding.PLAN_2D_FUSED, binding.PLAN_2D_ROWS_COLS
    for dt in (np.float32, np.float64, np.int32, np.uint16):
        assert binding.maxmin_plan_2d(dt, 3, 3) == F
        assert binding.maxmin_plan_2d(dt, 7, 257) == F and binding.maxmin_plan_2d(dt, 7, 258) == RC
        assert binding.maxmin_plan_2d(dt, 15, 129) == F and binding.maxmin_plan_2d(dt, 15, 130) == RC
        big = F if dt == np.uint16 else RC
        assert binding.maxmin_plan_2d(dt, 16, 65) == big and binding.maxmin_plan_2d(dt, 16, 66) == RC
        assert binding.maxmin_plan_2d(dt, 23, 65) == big and binding.maxmin_plan_2d(dt, 24, 65) == RC
        assert binding.maxmin_plan_2d(dt, 31, 65) == RC
        assert binding.maxmin_plan_2d(dt, 32, 3) == RC and binding.maxmin_plan_2d(dt, 63, 63) == RC
        assert binding.maxmin_plan_2d(dt, 65, 1) == RC
        # one output: the fused pass up to w_rows 15 for every type
        assert binding.maxmin_plan_2d(dt, 15, 65, outputs=1) == F
        assert binding.maxmin_plan_2d(dt, 16, 3, outputs=1) == RC
    monkeypatch.setenv("MAXMIN_2D_FUSED", "1")
    assert binding.maxmin_plan_2d(np.float32, 63, 63) == F
    monkeypatch.setenv("MAXMIN_2D_FUSED", "0")
    assert binding.maxmin_plan_2d(np.float32, 3, 3) == RC
    with pytest.raises(binding.MaxMinError):
        binding.maxmin_plan_2d(np.float32, 0, 3)
    with pytest.raises(binding.MaxMinError):
        binding.maxmin_plan_2d(np.float32, 3, 3, outputs=3)


def test_planner(lib):
    binding.maxmin_set_strategy(binding.STRATEGY_AUTO)
    assert binding.maxmin_plan(np.float32, 1 << 20, 64) == binding.STRATEGY_TILE
    assert binding.maxmin_plan(np.float32, 1 << 20, 1024) == binding.STRATEGY_TILE
    assert binding.maxmin_plan(np.float32, 1 << 20, 2048) == binding.STRATEGY_TILE
    assert binding.maxmin_plan(np.float32, 1 << 20, 2049) == binding.STRATEGY_TILE
    assert binding.maxmin_plan(np.float32, 1 << 20, 4096) == binding.STRATEGY_TILE
    assert binding.maxmin_plan(np.float32, 1 << 20, 4097) == binding.STRATEGY_TILE
    assert binding.maxmin_plan(np.float32, 1 << 20, 8192) == binding.STRATEGY_TILE
    assert binding.maxmin_plan(np.float32, 1 << 20, 8193) in (binding.STRATEGY_CHUNK, binding.STRATEGY_RUN)
    binding.maxmin_set_strategy(binding.STRATEGY_CHUNK)
    assert binding.maxmin_plan(np.float32, 1 << 20, 64) == binding.STRATEGY_CHUNK
    binding.maxmin_set_strategy(binding.STRATEGY_TILE)
    assert binding.maxmin_plan(np.float32, 1 << 20, 9000) in (binding.STRATEGY_CHUNK, binding.STRATEGY_RUN)  # tile cannot
    binding.maxmin_set_strategy(binding.STRATEGY_AUTO)


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    monkeypatch.setattr(binding, "LIB_PATH", str(tmp_path / "nope.so"))
    monkeypatch.setattr(binding, "_lib", None)
    with pytest.raises(RuntimeError, match="not built"):
        binding.lib()
