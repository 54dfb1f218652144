// C ABI of libmaxmin: argument checks, the planner, per-stream scratch
// memory, the batched graph cache and stream-state handles.  All compute is
// in the gfx950 kernels (mm_kernels_*.hip); nothing here touches values.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <initializer_list>
#include <map>
#include <mutex>
#include <string>
#include <vector>
#include <tuple>
#include <utility>

#include "maxmin.h"
#include "mm_launch.hpp"

namespace {

using mm::JobArgs;

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

int ok() {
  g_err.clear();
  return MAXMIN_OK;
}

int hip_fail(hipError_t e, const char* what) {
  return fail(MAXMIN_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

size_t dsize(int dt) {
  switch (dt) {
    case MAXMIN_F32: return 4;
    case MAXMIN_F64: return 8;
    case MAXMIN_I32: return 4;
    case MAXMIN_U16: return 2;
    default: return 0;
  }
}

bool aligned(const void* p, size_t s) { return ((uintptr_t)p % s) == 0; }

std::atomic<int> g_force{0};

// Launch parameters the planner uses, per dtype.  The defaults are the
// choices measured best on MI355X; maxmin_autotune re-measures them on the
// device at hand.  Environment variables still override (experiments).
// On MI355X (n = 2^28 float32) runs of 4 sub-tiles for w <= 2048 ran 4-5%
// faster than 16 (w = 16: 0.612 against 0.642 ms, w = 256: 0.648 against
// 0.674 ms); longer windows re-read up to four sub-tiles of halo per run
// and keep runs of 64 (16 sub-tiles there: 0.72 against 0.69 ms at 4096).
mm::BatchPlan default_plan() {
  mm::BatchPlan p{};
  for (int wc = 0; wc < mm::kBatchWClasses; ++wc)
    for (int nc = 0; nc < mm::kBatchNClasses; ++nc) p.strat[wc][nc] = wc < 3 ? mm::kBatchTile : mm::kBatchChunk;
  p.run_subtiles = 1;
  return p;
}
struct Tuning {
  int tile_run = 4;        // sub-tiles per run, single-series tile launches, w <= 2048
  int tile_run_long = 64;  // the same for 2048 < w <= 8192
  int rows_run = 16;       // sub-tiles per run, row pass of the 2-D filter
  int ranges_one = 16;     // chunk ticket ranges, one-chunk windows (w <= 4096; chunk strategy forced)
  int ranges_long = 0;     // chunk ticket ranges, longer windows on the look-back kernel
  int long_strategy = MAXMIN_STRATEGY_CHUNK;  // w > 8192: chunk or run
  mm::BatchPlan batch = default_plan();       // batched calls: strategy per size class, tile size
  int tuned = 0;
};
std::mutex g_tune_mu;
Tuning g_tune[4];
std::atomic<int64_t> g_tune_version{0};  // bumped on every change (keys the batched graph cache)
Tuning tuning(int dt) {
  std::lock_guard<std::mutex> g(g_tune_mu);
  return g_tune[dt >= 0 && dt < 4 ? dt : 0];
}

// The batched plan of `dt`, with the experiment overrides MAXMIN_BATCH_PLAN
// (tile / chunk: that strategy for every class it applies to) and
// MAXMIN_BATCH_RUN (tile size in sub-tiles).
mm::BatchPlan batch_plan(int dt) {
  mm::BatchPlan p = tuning(dt).batch;
  if (const char* e = getenv("MAXMIN_BATCH_PLAN")) {
    const int f = !strcmp(e, "chunk") ? mm::kBatchChunk : (!strcmp(e, "tile") ? mm::kBatchTile : -1);
    if (f >= 0)
      for (int wc = 0; wc < 3; ++wc)
        for (int nc = 0; nc < mm::kBatchNClasses; ++nc) p.strat[wc][nc] = (uint8_t)f;
  }
  if (const char* e = getenv("MAXMIN_BATCH_RUN")) {
    const int r = atoi(e);
    if (r >= 1 && r <= 64) p.run_subtiles = r;
  }
  return p;
}

int env_strategy() {
  static int v = -1;
  if (v < 0) {
    const char* e = getenv("MAXMIN_FORCE_STRATEGY");
    v = 0;
    if (e && (!strcmp(e, "tile") || !strcmp(e, "1"))) v = MAXMIN_STRATEGY_TILE;
    if (e && (!strcmp(e, "chunk") || !strcmp(e, "2"))) v = MAXMIN_STRATEGY_CHUNK;
    if (e && (!strcmp(e, "run") || !strcmp(e, "3"))) v = MAXMIN_STRATEGY_RUN;
  }
  return v;
}

// Chunks per run for the run strategy on a single series, and whether its
// warm-up (re-reading the K-1 chunks before each run) stays small.
int64_t run_chunks_per_run(int dt, int64_t n, int64_t w) {
  const int64_t nch = mm::crun_chunks(n, w);
  const int64_t cap = mm::grid_cap(dt, mm::kStratRun);
  return std::max<int64_t>(1, (nch + cap - 1) / cap);
}
// Planner: streaming tiles for w <= 8192, chunks with cross-workgroup
// look-back above.  Chunk runs are used only when forced: on MI355X with
// n = 2^28 float32 they ran slower than look-back chunks at w = 4096 and 8192
// (1.46 ms against 0.83 and 0.88 ms).
int plan_strategy(int dt, int64_t n, int64_t w) {
  (void)n;
  int f = g_force.load();
  if (!f) f = env_strategy();
  const bool run_ok = (w + mm::kCrMax - 1) / mm::kCrMax <= mm::kCrRing;
  if (f == MAXMIN_STRATEGY_CHUNK) return MAXMIN_STRATEGY_CHUNK;
  if (f == MAXMIN_STRATEGY_RUN && run_ok) return MAXMIN_STRATEGY_RUN;
  if (w <= mm::kTileMaxW4) return MAXMIN_STRATEGY_TILE;
  if (!f && run_ok && tuning(dt).long_strategy == MAXMIN_STRATEGY_RUN) return MAXMIN_STRATEGY_RUN;
  return MAXMIN_STRATEGY_CHUNK;
}

// The fused 2-D pass serves the windows it fits up to 15 rows (23 for
// 16-bit data with both outputs); past those its one column per lane and
// LDS ring of 2B rows lose to rows-then-columns with the streaming ring
// column pass.  On MI355X (8192^2, square windows, ms per call, fused /
// rows-then-columns): float32 w = 15 0.30 / 0.46, 16 0.45 / 0.42, 31 0.50
// / 0.45, 63 0.90 / 0.51; float32 max-only w = 15 0.17 / 0.26, 16 0.27 /
// 0.25, 31 0.29 / 0.27; uint16 w = 20 0.30 / 0.33, 24 0.31 / 0.31, 31 0.32
// / 0.30; uint16 max-only w = 15 0.11 / 0.22, 16 0.21 / 0.20.
// MAXMIN_2D_FUSED=0 / =1 force either path where both apply (experiments
// and tests).
bool fused_2d(int dtype, int64_t w_rows, int64_t w_cols, bool one_output) {
  if (!mm::f2d_eligible(dtype, w_rows, w_cols)) return false;
  const char* e = getenv("MAXMIN_2D_FUSED");
  if (e && !strcmp(e, "0")) return false;
  if (e && !strcmp(e, "1")) return true;
  return w_rows < (dsize(dtype) == 2 && !one_output ? 24 : 16);
}
// Column pass of rows-then-columns: the fused kernel's column filter alone
// (streaming down bands) for windows under 16 rows and for 16-bit data,
// else blocks of w_rows rows (on MI355X, 8192^2 float32, w = 31 / 63: 0.31
// / 0.47 ms against 0.50 / 0.87 ms for the streaming filter; uint16 w =
// 63: 0.80 against 0.45 ms the other way).
// Which column pass: 0 blocks of w_rows rows (launch_cols), 1 the fused
// kernel's streaming column filter, 2 the LDS-ring streaming pass.  From 16
// rows on the ring (MI355X, 8192^2, whole call: float32 w = 16 / 31 / 63
// 0.42 / 0.45 / 0.51 ms against 0.48 / 0.49 / 0.50 streaming and 0.51 /
// 0.49 / 0.53 blocks; uint16 0.29 / 0.30 / 0.32 against 0.30 / 0.32 /
// 0.42 streaming); below it the streaming filter (its ring of 2B rows is
// small there).  MAXMIN_COLS_PASS=block / stream / ring forces one where it
// applies (experiments, tests).
int cols_pass_2d(int dtype, int64_t w_rows) {
  const char* e = getenv("MAXMIN_COLS_PASS");
  if (e && !strcmp(e, "block")) return 0;
  if (e && !strcmp(e, "stream")) return 1;
  if (e && !strcmp(e, "ring")) return 2;
  if (dsize(dtype) != 8 && w_rows >= 16 && w_rows <= 64) return 2;
  return w_rows < 16 || (dsize(dtype) == 2 && w_rows <= 64) ? 1 : 0;
}

// Long windows of a single series (more than one chunk per block): the
// one-pass column kernel; the look-back chunk kernel only when
// MAXMIN_LONG_LOOKBACK=1 asks for it (experiments, tests).  On MI355X (n =
// 2^28 float32) the one-pass kernel matched or beat look-back everywhere
// (w = 16384 0.84 / 0.85 ms, 32768 0.85 / 0.91 ms) and the two passes
// (aggregates, then columns) everywhere (w = 8193 1.15 / 1.56 ms, 20000
// 0.77 / 0.90, 65536 0.77 / 0.94, 2^20 0.89 / 0.94).
// The two passes instead of the one-pass kernel: MAXMIN_LONG_ONEPASS=0
// (experiments, tests); also where a cooperative launch cannot hold one
// column group.
bool long_onepass() {
  const char* e = getenv("MAXMIN_LONG_ONEPASS");
  return !(e && !strcmp(e, "0"));
}

bool long_lookback(int64_t w) {
  (void)w;
  const char* e = getenv("MAXMIN_LONG_LOOKBACK");
  return e && !strcmp(e, "1");
}

// Which tile kernel a single series or a row pass of window w runs.
int tile_kind(int64_t w) {
  return w <= mm::kTileMaxW    ? mm::kStratTile
         : w <= mm::kTileMaxW2 ? mm::kStratTile2
         : w <= 3 * mm::kTileOut ? mm::kStratTile3
                                 : mm::kStratTile4;
}

// ------------------------------------------------------------ workspaces
typedef std::tuple<int, const void*, const void*, const void*, const void*, int64_t, void*, void*, std::string> GraphKey;

struct Workspace {
  int device = 0;
  hipStream_t stream = nullptr;
  mm::Ctl* ctl = nullptr;
  uint64_t* ring = nullptr;
  uint32_t ring_lg = 0;
  void* descs = nullptr;
  int64_t desc_cap = 0;
  int64_t* pre = nullptr;  // 2 * pre_cap + 2 * kBatchMaxGroups + 2 int64
  int64_t pre_cap = 0;
  void* tmp = nullptr;
  size_t tmp_bytes = 0;
  void* tmp2 = nullptr;  // morphology: the first filter's image
  size_t tmp2_bytes = 0;
  void* env = nullptr;  // batched envelopes: windows [S] and output offsets [S+1]
  size_t env_bytes = 0;
  void* agg = nullptr;  // long windows: chunk maxima and minima
  size_t agg_bytes = 0;
  uint64_t* rec = nullptr;  // long windows, one pass: tagged chunk records (zeroed when allocated)
  size_t rec_bytes = 0;
  std::map<GraphKey, hipGraphExec_t> graphs;
};

std::mutex g_mu;
std::map<std::pair<int, hipStream_t>, Workspace*> g_ws;

bool capturing(hipStream_t s) {
  if (!s) return false;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &cs) != hipSuccess) return false;
  return cs != hipStreamCaptureStatusNone;
}

void drop_graphs(Workspace* ws) {
  for (auto& kv : ws->graphs) hipGraphExecDestroy(kv.second);
  ws->graphs.clear();
}

// Any growth of scratch memory happens outside graph capture: it allocates
// and initialises synchronously.
int grow_guard(Workspace* ws, const char* what) {
  if (capturing(ws->stream))
    return fail(MAXMIN_EBUSY, "%s: scratch memory must grow while the stream is being captured; "
                              "run the same call once before capturing", what);
  hipError_t e = ws->stream ? hipStreamSynchronize(ws->stream) : hipDeviceSynchronize();
  if (e != hipSuccess) return hip_fail(e, what);
  drop_graphs(ws);
  return MAXMIN_OK;
}

int get_ws(hipStream_t s, Workspace** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  std::lock_guard<std::mutex> g(g_mu);
  auto key = std::make_pair(dev, s);
  auto it = g_ws.find(key);
  if (it != g_ws.end()) {
    *out = it->second;
    return MAXMIN_OK;
  }
  Workspace* ws = new Workspace;
  ws->device = dev;
  ws->stream = s;
  if (capturing(s)) {
    delete ws;
    return fail(MAXMIN_EBUSY, "first use of a stream must not be inside graph capture");
  }
  e = hipMalloc((void**)&ws->ctl, sizeof(mm::Ctl));
  if (e != hipSuccess) {
    delete ws;
    return fail(MAXMIN_ENOMEM, "hipMalloc(control words): %s", hipGetErrorString(e));
  }
  mm::Ctl init{};
  init.epoch = 1u;
  e = hipMemcpy(ws->ctl, &init, sizeof init, hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    hipFree(ws->ctl);
    delete ws;
    return hip_fail(e, "hipMemcpy(control words)");
  }
  g_ws[key] = ws;
  *out = ws;
  return MAXMIN_OK;
}

constexpr uint32_t kRingMaxLg = 20;  // 2^20 records (32 MiB); larger launches lap the ring

int ensure_ring(Workspace* ws, int64_t ntiles) {
  uint32_t lg = 10;
  while (lg < kRingMaxLg && (int64_t(1) << lg) < ntiles) ++lg;
  if (ws->ring && ws->ring_lg >= lg) return MAXMIN_OK;
  int r = grow_guard(ws, "look-back records");
  if (r) return r;
  if (ws->ring) hipFree(ws->ring);
  ws->ring = nullptr;
  const size_t bytes = (size_t)4 * sizeof(uint64_t) << lg;
  hipError_t e = hipMalloc((void**)&ws->ring, bytes);
  if (e != hipSuccess) return fail(MAXMIN_ENOMEM, "hipMalloc(look-back records, %zu B): %s", bytes, hipGetErrorString(e));
  e = hipMemset(ws->ring, 0, bytes);  // tag 0 never validates
  if (e != hipSuccess) return hip_fail(e, "hipMemset(look-back records)");
  e = hipDeviceSynchronize();
  if (e != hipSuccess) return hip_fail(e, "hipDeviceSynchronize");
  ws->ring_lg = lg;
  return MAXMIN_OK;
}

int ensure_batch(Workspace* ws, int64_t S) {
  if (ws->descs && ws->desc_cap >= S && ws->pre_cap >= mm::batch_pre_len(S)) return MAXMIN_OK;
  int r = grow_guard(ws, "batched descriptors");
  if (r) return r;
  if (ws->descs) hipFree(ws->descs);
  if (ws->pre) hipFree(ws->pre);
  ws->descs = nullptr;
  ws->pre = nullptr;
  const int64_t cap = std::max<int64_t>(S, 1024);
  hipError_t e = hipMalloc(&ws->descs, (size_t)cap * mm::series_bytes());
  // one prefix array of cap + 1 per path, then the setup's per-workgroup totals
  if (e == hipSuccess) e = hipMalloc((void**)&ws->pre, (size_t)mm::batch_pre_len(cap) * sizeof(int64_t));
  if (e != hipSuccess) return fail(MAXMIN_ENOMEM, "hipMalloc(batched descriptors): %s", hipGetErrorString(e));
  ws->desc_cap = cap;
  ws->pre_cap = mm::batch_pre_len(cap);
  return MAXMIN_OK;
}

int ensure_buf(Workspace* ws, void** buf, size_t* have, size_t bytes) {
  if (*buf && *have >= bytes) return MAXMIN_OK;
  int r = grow_guard(ws, "scratch buffers");
  if (r) return r;
  if (*buf) hipFree(*buf);
  *buf = nullptr;
  hipError_t e = hipMalloc(buf, bytes);
  if (e != hipSuccess) return fail(MAXMIN_ENOMEM, "hipMalloc(scratch, %zu B): %s", bytes, hipGetErrorString(e));
  *have = bytes;
  return MAXMIN_OK;
}
int ensure_tmp(Workspace* ws, size_t bytes) { return ensure_buf(ws, &ws->tmp, &ws->tmp_bytes, bytes); }
// Record buffer of the one-pass long-window kernel: zeroed when allocated
// (tag 0 never validates; every later record carries a launch epoch).
int ensure_rec(Workspace* ws, size_t bytes) {
  if (ws->rec && ws->rec_bytes >= bytes) return MAXMIN_OK;
  void* p = ws->rec;
  int r = ensure_buf(ws, &p, &ws->rec_bytes, bytes);
  ws->rec = (uint64_t*)p;
  if (r) return r;
  hipError_t e = hipMemset(ws->rec, 0, bytes);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) return hip_fail(e, "hipMemset(long-window records)");
  return MAXMIN_OK;
}
int ensure_tmp2(Workspace* ws, size_t bytes) { return ensure_buf(ws, &ws->tmp2, &ws->tmp2_bytes, bytes); }

// Ticket ranges for a single-series chunk launch (0, 1, 8, 16 or 32), for
// one-chunk windows (w <= 4096) and for longer ones; the environment
// variables MAXMIN_CHUNK_RANGES and MAXMIN_CHUNK_RANGES_LONG override them.
int chunk_ranges(int dt, int64_t w) {
  const bool one = w <= mm::kChunkMax;
  const Tuning t = tuning(dt);
  int v = one ? t.ranges_one : t.ranges_long;
  const char* e = getenv(one ? "MAXMIN_CHUNK_RANGES" : "MAXMIN_CHUNK_RANGES_LONG");
  if (e) {
    const int x = atoi(e);
    if (x == 0 || x == 1 || x == 8 || x == 16 || x == 32) v = x;
  }
  return v;
}

}  // namespace

namespace mm {
// One series with the tile kernel (w <= 8192): run length from the tuning
// table, persistent grid; no scratch memory.
hipError_t launch_tile_series(int dt, JobArgs a, hipStream_t st) {
  const int ks = tile_kind(a.w);
  const int cap = grid_cap(dt, ks);
  // a run re-reads the w-1 inputs after it: runs 4x longer for windows
  // over more than one sub-tile (MI355X, n = 2^28 float32, w =
  // 2049..4096: 64 sub-tiles 0.71-0.73 ms, 32: 0.72-0.73, 16: 0.74-0.75)
  const Tuning t = tuning(dt);
  const int64_t rmax = (int64_t)(ks == kStratTile ? t.tile_run : t.tile_run_long) * kTileOut;
  a.run = run_length(a.n - a.w + 1, cap, rmax);
  if (const char* e = getenv("MAXMIN_TILE_RUN")) {
    const int64_t r = atoll(e) / kTileOut * kTileOut;
    if (r > 0 && r < a.run) a.run = r;
  }
  a.ntiles = run_count(a.n, a.w, a.run);
  const int grid = (int)std::min<int64_t>(a.ntiles, cap);
  return launch_1d(dt, ks, a, grid, st);
}
}  // namespace mm

namespace {

// Run one 1-D series (plain call or stream push) with the planned strategy.
int run_series(int dt, JobArgs a, hipStream_t st, const char* what) {
  const int strat = plan_strategy(dt, a.n, a.w);
  hipError_t e;
  if (strat == MAXMIN_STRATEGY_TILE) {
    e = mm::launch_tile_series(dt, a, st);
  } else if (strat == MAXMIN_STRATEGY_RUN) {
    a.run = run_chunks_per_run(dt, a.n, a.w);
    a.ntiles = (mm::crun_chunks(a.n, a.w) + a.run - 1) / a.run;
    const int grid = (int)std::min<int64_t>(a.ntiles, mm::grid_cap(dt, mm::kStratRun));
    e = mm::launch_1d(dt, mm::kStratRun, a, grid, st);
  } else if (a.w > mm::kChunkMax && !long_lookback(a.w)) {
    // more than one chunk per block: chunk aggregates, then columns of
    // chunks (no look-back, the chunk w back kept in registers)
    Workspace* ws = nullptr;
    int r = get_ws(st, &ws);
    if (r) return r;
    e = hipErrorNotSupported;
    if (long_onepass()) {
      if ((r = ensure_rec(ws, (size_t)std::max<int64_t>(1, mm::long1_records(dt, a.n, a.w)) * 32))) return r;
      e = mm::launch_long1(dt, a, ws->rec, ws->ctl, st);
    }
    if (e == hipErrorNotSupported) {
      const int64_t nch = mm::chunk_count(a.n, a.w, mm::long_chunk_max(a.w));
      if ((r = ensure_buf(ws, &ws->agg, &ws->agg_bytes, (size_t)std::max<int64_t>(1, 2 * nch) * dsize(dt)))) return r;
      e = mm::launch_long(dt, a, ws->agg, st);
    }
  } else {
    Workspace* ws = nullptr;
    int r = get_ws(st, &ws);
    if (r) return r;
    a.ntiles = mm::chunk_count(a.n, a.w);
    r = ensure_ring(ws, a.ntiles);
    if (r) return r;
    a.ring = ws->ring;
    a.ring_lg = ws->ring_lg;
    a.ctl = ws->ctl;
    a.ranges = chunk_ranges(dt, a.w);
    const int grid = (int)std::min<int64_t>(a.ntiles, mm::grid_cap(dt, mm::kStratChunk));
    e = mm::launch_1d(dt, mm::kStratChunk, a, grid, st);
  }
  if (e != hipSuccess) return hip_fail(e, what);
  return ok();
}

bool g_graphs_enabled() {
  static int v = -1;
  if (v < 0) {
    const char* e = getenv("MAXMIN_BATCHED_GRAPHS");
    v = (e && !strcmp(e, "0")) ? 0 : 1;
  }
  return v == 1;
}

}  // namespace

namespace mm {
// Look-back state of `stream` (control words and a ring of at least
// min(ntiles, 2^20) records), for launches made outside this file.
int stream_lookback_state(hipStream_t stream, int64_t ntiles, uint64_t** ring, uint32_t* lg, Ctl** ctl) {
  Workspace* ws = nullptr;
  int r = get_ws(stream, &ws);
  if (r) return r;
  if ((r = ensure_ring(ws, ntiles))) return r;
  *ring = ws->ring;
  *lg = ws->ring_lg;
  *ctl = ws->ctl;
  return MAXMIN_OK;
}
int set_error(int code, const char* msg) { return fail(code, "%s", msg); }
BatchPlan batch_plan_for(int dtype) { return batch_plan(dtype); }
int long_col_v_override() {
  static const int v = [] {
    const char* e = getenv("MAXMIN_LONG_V");
    return e && !strcmp(e, "8") ? 8 : (e && !strcmp(e, "16") ? 16 : 0);
  }();
  return v;
}
}  // namespace mm

struct maxmin_stream {
  int dt;
  int64_t w;
  int64_t t;
  int device;
  void* carry[2];
  int cur;
  hipEvent_t last;  // recorded after each push: destroy waits for it, not for the device
};

extern "C" {

const char* maxmin_last_error(void) { return g_err.c_str(); }

const char* maxmin_version(void) { return "maxmin-gfx950 0.1"; }

int maxmin_set_strategy(int strategy) {
  if (strategy < MAXMIN_STRATEGY_AUTO || strategy > MAXMIN_STRATEGY_RUN)
    return fail(MAXMIN_EINVAL, "maxmin_set_strategy: unknown strategy %d", strategy);
  g_force.store(strategy);
  return ok();
}

int maxmin_plan(int dtype, int64_t n, int64_t w) { return plan_strategy(dtype, n, w); }

int maxmin_plan_2d(int dtype, int64_t w_rows, int64_t w_cols, int outputs) {
  if (!dsize(dtype)) return fail(MAXMIN_EINVAL, "maxmin_plan_2d: unknown dtype %d", dtype);
  if (w_rows < 1 || w_cols < 1) return fail(MAXMIN_EINVAL, "maxmin_plan_2d: window < 1");
  if (outputs != 1 && outputs != 2) return fail(MAXMIN_EINVAL, "maxmin_plan_2d: outputs=%d (1 or 2)", outputs);
  return fused_2d(dtype, w_rows, w_cols, outputs == 1) ? MAXMIN_2D_FUSED : MAXMIN_2D_ROWS_COLS;
}

int maxmin_filter(int dtype, const void* d_in, int64_t n, int64_t w, void* d_max, void* d_min, void* stream) {
  const size_t s = dsize(dtype);
  if (!s) return fail(MAXMIN_EINVAL, "maxmin_filter: unknown dtype %d", dtype);
  if (w < 1) return fail(MAXMIN_EINVAL, "maxmin_filter: window w=%lld < 1", (long long)w);
  if (n < 0) return fail(MAXMIN_EINVAL, "maxmin_filter: n=%lld < 0", (long long)n);
  if (n < w) return ok();  // no complete window
  if (!d_in || (!d_max && !d_min)) return fail(MAXMIN_EINVAL, "maxmin_filter: null pointer");
  if (!aligned(d_in, s) || !aligned(d_max, s) || !aligned(d_min, s))
    return fail(MAXMIN_EINVAL, "maxmin_filter: pointer not aligned to the element size");
  JobArgs a;
  a.mode = 0;
  a.a = d_in;
  a.na = n;
  a.n = n;
  a.w = w;
  a.omax = d_max;
  a.omin = d_min;
  return run_series(dtype, a, (hipStream_t)stream, "maxmin_filter");
}

int maxmin_argfilter(int dtype, const void* d_in, int64_t n, int64_t w, void* d_max, void* d_min, int64_t* d_argmax,
                     int64_t* d_argmin, void* stream) {
  const size_t s = dsize(dtype);
  if (!s) return fail(MAXMIN_EINVAL, "maxmin_argfilter: unknown dtype %d", dtype);
  if (w < 1) return fail(MAXMIN_EINVAL, "maxmin_argfilter: window w=%lld < 1", (long long)w);
  if (n < 0) return fail(MAXMIN_EINVAL, "maxmin_argfilter: n=%lld < 0", (long long)n);
  if (n < w) return ok();  // no complete window
  if (!d_in || !d_max || !d_min || !d_argmax || !d_argmin) return fail(MAXMIN_EINVAL, "maxmin_argfilter: null pointer");
  if (!aligned(d_in, s) || !aligned(d_max, s) || !aligned(d_min, s) || !aligned(d_argmax, 8) || !aligned(d_argmin, 8))
    return fail(MAXMIN_EINVAL, "maxmin_argfilter: pointer not aligned to the element size");
  hipStream_t st = (hipStream_t)stream;
  // 4096 < w <= 2^29: per-chunk aggregates, then columns of chunks (the
  // input read twice, each output written once).  MAXMIN_ARG_CHUNK=0 keeps
  // the level-array paths below (tests).
  {
    const char* eh = getenv("MAXMIN_ARG_CHUNK");
    if (w > mm::kTileMaxW2 && w <= (int64_t(1) << 29) && !(eh && !strcmp(eh, "0"))) {
      Workspace* ws = nullptr;
      int r = get_ws(st, &ws);
      if (r) return r;
      if ((r = ensure_tmp(ws, mm::arg_chunk_scratch(dtype, n, w)))) return r;
      hipError_t e = mm::launch_arg_chunks(dtype, d_in, n, w, ws->tmp, d_max, d_argmax, d_min, d_argmin, st);
      if (e != hipSuccess) return hip_fail(e, "maxmin_argfilter (chunks)");
      return ok();
    }
  }
  // 2 x 4096 < w <= 31 x 4096: the tile kernel at q = floor(w / F), F =
  // ceil(w / 4096), then one running window of F rows of q level entries
  // (each entry read once).  On MI355X (n = 2^28 float32) it beat the
  // combine steps below from F = 3 on (w = 8193 / 16385 / 65536: 6.1 / 6.3
  // / 5.3 ms against 6.6 / 8.7 / 13.1 ms) and lost at F = 2 (w = 4097: 6.1
  // against 5.5 ms).  MAXMIN_ARG_CHAIN=1 forces the combine steps (tests).
  if (w > 2 * mm::kTileMaxW2) {
    const int64_t F = (w + mm::kTileMaxW2 - 1) / mm::kTileMaxW2;
    const char* ec = getenv("MAXMIN_ARG_CHAIN");
    if (F <= mm::kArgColsMaxF && !(ec && !strcmp(ec, "1"))) {
      const int64_t q = w / F;
      const size_t set_bytes = (size_t)n * (2 * s + 2 * sizeof(int64_t));
      Workspace* ws = nullptr;
      int r = get_ws(st, &ws);
      if (r) return r;
      if ((r = ensure_tmp(ws, set_bytes))) return r;
      char* lv = (char*)ws->tmp;
      void* lvx = lv;
      void* lvn = lv + (size_t)n * s;
      int64_t* lix = (int64_t*)(lv + (size_t)n * 2 * s);
      int64_t* lin = lix + n;
      JobArgs a;
      a.mode = 0;
      a.a = d_in;
      a.na = n;
      a.n = n;
      a.w = q;
      a.omax = lvx;
      a.omin = lvn;
      a.amax = lix;
      a.amin = lin;
      const int ks = q <= mm::kTileMaxW ? mm::kStratArg : mm::kStratArg2;
      const int cap = mm::grid_cap(dtype, ks);
      a.run = mm::run_length(n - q + 1, cap, (ks == mm::kStratArg2 ? 4 : 1) * mm::kTileRunMax);
      a.ntiles = mm::run_count(n, q, a.run);
      hipError_t e = mm::launch_1d(dtype, ks, a, (int)std::min<int64_t>(a.ntiles, cap), st);
      if (e != hipSuccess) return hip_fail(e, "maxmin_argfilter");
      e = mm::launch_arg_cols(dtype, lvx, lix, lvn, lin, n - q + 1, q, w, n - w + 1, d_max, d_argmax, d_min, d_argmin,
                              st);
      if (e != hipSuccess) return hip_fail(e, "maxmin_argfilter (rows of level entries)");
      return ok();
    }
  }
  // windows: w, then ceil(w/F), ... down to the first one the tile kernel
  // takes, with the fewest steps of fan-in F <= 16 (each step reads F
  // shorter windows per output)
  int L = 0;
  for (int64_t p = w; p > mm::kTileMaxW2; p = (p + 15) / 16) ++L;
  int F = 1;
  if (L > 0) {
    // the smallest F whose L-th power reaches w / kTileMaxW2
    F = 2;
    for (;;) {
      int64_t p = w;
      for (int l = 0; l < L; ++l) p = (p + F - 1) / F;
      if (p <= mm::kTileMaxW2) break;
      ++F;
    }
  }
  std::vector<int64_t> chain{w};
  for (int l = 0; l < L; ++l) chain.push_back((chain.back() + F - 1) / F);
  std::reverse(chain.begin(), chain.end());
  // level buffers: values (max, min) and locations (max, min), two sets
  char* set[2] = {nullptr, nullptr};
  const size_t set_bytes = (size_t)n * (2 * s + 2 * sizeof(int64_t));
  if (L > 0) {
    Workspace* ws = nullptr;
    int r = get_ws(st, &ws);
    if (r) return r;
    if ((r = ensure_tmp(ws, (L > 1 ? 2 : 1) * set_bytes))) return r;
    set[0] = (char*)ws->tmp;
    set[1] = (char*)ws->tmp + (L > 1 ? set_bytes : 0);
  }
  auto vx = [&](int k) -> void* { return set[k]; };
  auto vn = [&](int k) -> void* { return set[k] + (size_t)n * s; };
  auto ix = [&](int k) -> int64_t* { return (int64_t*)(set[k] + (size_t)n * 2 * s); };
  auto in = [&](int k) -> int64_t* { return (int64_t*)(set[k] + (size_t)n * (2 * s + sizeof(int64_t))); };
  // level 0: the tile kernel with locations
  JobArgs a;
  a.mode = 0;
  a.a = d_in;
  a.na = n;
  a.n = n;
  a.w = chain[0];
  a.omax = L ? vx(0) : d_max;
  a.omin = L ? vn(0) : d_min;
  a.amax = L ? ix(0) : d_argmax;
  a.amin = L ? in(0) : d_argmin;
  const int ks = a.w <= mm::kTileMaxW ? mm::kStratArg : mm::kStratArg2;
  const int cap = mm::grid_cap(dtype, ks);
  a.run = mm::run_length(n - a.w + 1, cap, (ks == mm::kStratArg2 ? 4 : 1) * mm::kTileRunMax);
  a.ntiles = mm::run_count(n, a.w, a.run);
  hipError_t e = mm::launch_1d(dtype, ks, a, (int)std::min<int64_t>(a.ntiles, cap), st);
  if (e != hipSuccess) return hip_fail(e, "maxmin_argfilter");
  for (int l = 1; l <= L; ++l) {
    const int src = (l - 1) & 1, dst = l & 1;
    const bool last = l == L;
    const int64_t q = chain[l - 1], p = chain[l];
    e = mm::launch_arg_combine(dtype, vx(src), vn(src), ix(src), in(src), q, p, (int)((p + q - 1) / q),
                               n - p + 1, last ? d_max : vx(dst), last ? d_min : vn(dst), last ? d_argmax : ix(dst),
                               last ? d_argmin : in(dst), st);
    if (e != hipSuccess) return hip_fail(e, "maxmin_argfilter (combine)");
  }
  return ok();
}

int maxmin_out_offsets(const int64_t* h_in_offsets, const int64_t* h_windows, int64_t S, int64_t* h_out_offsets) {
  if (S < 0) return fail(MAXMIN_EINVAL, "maxmin_out_offsets: S < 0");
  if (!h_in_offsets || !h_out_offsets || (S > 0 && !h_windows))
    return fail(MAXMIN_EINVAL, "maxmin_out_offsets: null pointer");
  h_out_offsets[0] = 0;
  for (int64_t k = 0; k < S; ++k) {
    const int64_t n = h_in_offsets[k + 1] - h_in_offsets[k];
    if (n < 0) return fail(MAXMIN_EINVAL, "maxmin_out_offsets: offsets decrease at series %lld", (long long)k);
    if (h_windows[k] < 1) return fail(MAXMIN_EINVAL, "maxmin_out_offsets: window < 1 at series %lld", (long long)k);
    h_out_offsets[k + 1] = h_out_offsets[k] + std::max<int64_t>(0, n - h_windows[k] + 1);
  }
  return ok();
}

int maxmin_filter_batched(int dtype, const void* d_in, const int64_t* d_in_offsets, const int64_t* d_windows,
                          const int64_t* d_out_offsets, int64_t S, void* d_max, void* d_min, void* stream) {
  const size_t s = dsize(dtype);
  if (!s) return fail(MAXMIN_EINVAL, "maxmin_filter_batched: unknown dtype %d", dtype);
  if (S < 0) return fail(MAXMIN_EINVAL, "maxmin_filter_batched: S < 0");
  if (S == 0) return ok();
  if (!d_in || !d_in_offsets || !d_windows || !d_out_offsets || (!d_max && !d_min))
    return fail(MAXMIN_EINVAL, "maxmin_filter_batched: null pointer");
  if (!aligned(d_in, s) || !aligned(d_max, s) || !aligned(d_min, s))
    return fail(MAXMIN_EINVAL, "maxmin_filter_batched: pointer not aligned to the element size");
  hipStream_t st = (hipStream_t)stream;
  Workspace* ws = nullptr;
  int r = get_ws(st, &ws);
  if (r) return r;
  if ((r = ensure_batch(ws, S))) return r;
  if ((r = ensure_ring(ws, int64_t(1) << kRingMaxLg))) return r;

  // One launch per path: the tile kernel of each lag (each workgroup
  // streams a contiguous range of its tiles, series by series, so the tile
  // size only sets how evenly the ranges split) and the chunk kernel; the
  // path of every series comes from the plan's strategy for its size class.
  const mm::BatchPlan plan = batch_plan(dtype);
  auto enqueue = [&]() -> hipError_t {
    int64_t* pre = ws->pre;
    hipError_t e = mm::launch_batched_setup(dtype, d_in, d_in_offsets, d_windows, d_out_offsets, S, d_max, d_min,
                                            ws->descs, pre, plan, st);
    if (e != hipSuccess) return e;
    JobArgs a;
    a.mode = 1;
    a.descs = ws->descs;
    a.S = S;
    a.run = (int64_t)plan.run_subtiles * mm::kTileOut;
    static const int kinds[4] = {mm::kStratTile, mm::kStratTile2, mm::kStratTile3, mm::kStratTile4};
    for (int p = 0; p < 4; ++p) {
      a.pre = pre + p * (S + 1);
      e = mm::launch_1d(dtype, kinds[p], a, mm::grid_cap(dtype, kinds[p]), st);
      if (e != hipSuccess) return e;
    }
    a.pre = pre + mm::kBatchChunkPath * (S + 1);
    a.ring = ws->ring;
    a.ring_lg = ws->ring_lg;
    a.ctl = ws->ctl;
    return mm::launch_1d(dtype, mm::kStratChunk, a, mm::grid_cap(dtype, mm::kStratChunk), st);
  };

  if (!st || !g_graphs_enabled() || capturing(st)) {
    hipError_t e = enqueue();
    if (e != hipSuccess) return hip_fail(e, "maxmin_filter_batched");
    return ok();
  }
  // replay a captured graph of the three launches when the same call repeats
  GraphKey key(dtype, d_in, d_in_offsets, d_windows, d_out_offsets, S, d_max, d_min,
               std::string((const char*)&plan, sizeof plan));
  auto it = ws->graphs.find(key);
  if (it == ws->graphs.end()) {
    hipError_t e = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
    hipError_t e1 = enqueue();
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(st, &g);
    if (e1 != hipSuccess) {
      if (g) hipGraphDestroy(g);
      return hip_fail(e1, "maxmin_filter_batched (capture)");
    }
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    hipGraphExec_t ex = nullptr;
    e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    hipGraphDestroy(g);
    if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
    if (ws->graphs.size() >= 64) drop_graphs(ws);
    it = ws->graphs.emplace(key, ex).first;
  }
  hipError_t e = hipGraphLaunch(it->second, st);
  if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
  return ok();
}

int maxmin_stream_create(int dtype, int64_t w, maxmin_stream_t** out) {
  const size_t s = dsize(dtype);
  if (!out) return fail(MAXMIN_EINVAL, "maxmin_stream_create: null out");
  *out = nullptr;
  if (!s) return fail(MAXMIN_EINVAL, "maxmin_stream_create: unknown dtype %d", dtype);
  if (w < 1) return fail(MAXMIN_EINVAL, "maxmin_stream_create: window w=%lld < 1", (long long)w);
  maxmin_stream* st = new maxmin_stream;
  st->dt = dtype;
  st->w = w;
  st->t = 0;
  st->cur = 0;
  hipGetDevice(&st->device);
  const size_t bytes = (size_t)std::max<int64_t>(1, w - 1) * s;
  st->carry[0] = st->carry[1] = nullptr;
  st->last = nullptr;
  hipError_t e = hipMalloc(&st->carry[0], bytes);
  if (e == hipSuccess) e = hipMalloc(&st->carry[1], bytes);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&st->last, hipEventDisableTiming);
  if (e != hipSuccess) {
    if (st->carry[0]) hipFree(st->carry[0]);
    if (st->carry[1]) hipFree(st->carry[1]);
    delete st;
    return fail(MAXMIN_ENOMEM, "maxmin_stream_create: hipMalloc(carry, %zu B): %s", bytes, hipGetErrorString(e));
  }
  *out = st;
  return ok();
}

int maxmin_stream_push(maxmin_stream_t* st, const void* d_chunk, int64_t m, void* d_max, void* d_min,
                       int64_t* h_n_out, void* stream) {
  if (!st) return fail(MAXMIN_EINVAL, "maxmin_stream_push: null handle");
  if (m < 0) return fail(MAXMIN_EINVAL, "maxmin_stream_push: m < 0");
  const int64_t c = std::min(st->t, st->w - 1);  // carried samples
  const int64_t total = c + m;
  const int64_t nout = std::max<int64_t>(0, total - st->w + 1);
  if (h_n_out) *h_n_out = 0;
  if (m == 0) return ok();
  const size_t s = dsize(st->dt);
  if (!d_chunk || (nout > 0 && !d_max && !d_min)) return fail(MAXMIN_EINVAL, "maxmin_stream_push: null pointer");
  if (!aligned(d_chunk, s) || (nout > 0 && (!aligned(d_max, s) || !aligned(d_min, s))))
    return fail(MAXMIN_EINVAL, "maxmin_stream_push: pointer not aligned to the element size");
  JobArgs a;
  a.mode = 0;
  a.a = st->carry[st->cur];
  a.na = c;
  a.b = d_chunk;
  a.n = total;
  a.w = st->w;
  a.omax = d_max;
  a.omin = d_min;
  a.carry = st->w > 1 ? st->carry[1 - st->cur] : nullptr;
  hipStream_t hs = (hipStream_t)stream;
  if (nout > 0) {
    int r = run_series(st->dt, a, hs, "maxmin_stream_push");
    if (r) return r;
  } else if (a.carry) {
    hipError_t e = mm::launch_carry_only(st->dt, a, hs);
    if (e != hipSuccess) return hip_fail(e, "maxmin_stream_push (carry)");
  }
  hipError_t e = hipEventRecord(st->last, hs);
  if (e != hipSuccess) return hip_fail(e, "maxmin_stream_push (event)");
  st->cur = 1 - st->cur;
  st->t += m;
  if (h_n_out) *h_n_out = nout;
  return ok();
}

int64_t maxmin_stream_samples(const maxmin_stream_t* st) { return st ? st->t : -1; }

// A stream's whole state is (t, its last min(t, w-1) samples): export copies
// it out after the handle's last push has finished; import builds a handle
// that continues from it (on the current device).
int maxmin_stream_export(const maxmin_stream_t* st, void* h_carry, int64_t* h_t) {
  if (!st || !h_t) return fail(MAXMIN_EINVAL, "maxmin_stream_export: null handle or h_t");
  const int64_t c = std::min(st->t, st->w - 1);
  if (c > 0 && !h_carry) return fail(MAXMIN_EINVAL, "maxmin_stream_export: null h_carry");
  hipError_t e = hipEventSynchronize(st->last);
  if (e == hipSuccess && c > 0) e = hipMemcpy(h_carry, st->carry[st->cur], (size_t)c * dsize(st->dt), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(e, "maxmin_stream_export");
  *h_t = st->t;
  return ok();
}

int maxmin_stream_import(int dtype, int64_t w, int64_t t, const void* h_carry, maxmin_stream_t** out) {
  if (!out) return fail(MAXMIN_EINVAL, "maxmin_stream_import: null out");
  *out = nullptr;
  if (!dsize(dtype)) return fail(MAXMIN_EINVAL, "maxmin_stream_import: unknown dtype %d", dtype);
  if (w < 1) return fail(MAXMIN_EINVAL, "maxmin_stream_import: window w=%lld < 1", (long long)w);
  if (t < 0) return fail(MAXMIN_EINVAL, "maxmin_stream_import: t=%lld < 0", (long long)t);
  const int64_t c = std::min(t, w - 1);
  if (c > 0 && !h_carry) return fail(MAXMIN_EINVAL, "maxmin_stream_import: null h_carry");
  maxmin_stream_t* st = nullptr;
  int r = maxmin_stream_create(dtype, w, &st);
  if (r) return r;
  if (c > 0) {
    const hipError_t e = hipMemcpy(st->carry[st->cur], h_carry, (size_t)c * dsize(dtype), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
      maxmin_stream_destroy(st);
      return hip_fail(e, "maxmin_stream_import");
    }
  }
  st->t = t;
  *out = st;
  return ok();
}

int maxmin_stream_destroy(maxmin_stream_t* st) {
  if (!st) return ok();
  // the carries may still be read or written by the last push: wait for it
  // (the event recorded after it), not for the whole device
  hipError_t e = hipEventSynchronize(st->last);
  hipFree(st->carry[0]);
  hipFree(st->carry[1]);
  hipEventDestroy(st->last);
  delete st;
  if (e != hipSuccess) return hip_fail(e, "maxmin_stream_destroy");
  return ok();
}

int maxmin_filter_2d(int dtype, const void* d_in, int64_t rows, int64_t cols, int64_t ld_in, int64_t w_rows,
                     int64_t w_cols, void* d_max, void* d_min, int64_t ld_out, void* stream) {
  const size_t s = dsize(dtype);
  if (!s) return fail(MAXMIN_EINVAL, "maxmin_filter_2d: unknown dtype %d", dtype);
  if (w_rows < 1 || w_cols < 1) return fail(MAXMIN_EINVAL, "maxmin_filter_2d: window < 1");
  if (rows < 0 || cols < 0) return fail(MAXMIN_EINVAL, "maxmin_filter_2d: negative size");
  if (ld_in < cols) return fail(MAXMIN_EINVAL, "maxmin_filter_2d: ld_in < cols");
  const int64_t orows = rows - w_rows + 1, oc = cols - w_cols + 1;
  if (orows <= 0 || oc <= 0) return ok();
  if (ld_out < oc) return fail(MAXMIN_EINVAL, "maxmin_filter_2d: ld_out < output width");
  if (!d_in || (!d_max && !d_min)) return fail(MAXMIN_EINVAL, "maxmin_filter_2d: null pointer");
  if (!aligned(d_in, s) || !aligned(d_max, s) || !aligned(d_min, s))
    return fail(MAXMIN_EINVAL, "maxmin_filter_2d: pointer not aligned to the element size");
  hipStream_t st = (hipStream_t)stream;
  // one fused pass when the windows fit it (no intermediate images)
  if (fused_2d(dtype, w_rows, w_cols, !d_max || !d_min)) {
    const char* eb = getenv("MAXMIN_2D_BAND");
    hipError_t e = mm::launch_f2d(dtype, d_in, ld_in, rows, cols, w_rows, w_cols, d_max, d_min, ld_out,
                                  eb ? atoll(eb) : 0, st);
    if (e == hipSuccess) return ok();
    if (e != hipErrorNotSupported) return hip_fail(e, "maxmin_filter_2d (fused)");
  }
  if ((orows + w_rows - 1) / w_rows > 65535)
    return fail(MAXMIN_EUNSUPPORTED, "maxmin_filter_2d: too many row blocks for one launch");
  Workspace* ws = nullptr;
  int r = get_ws(st, &ws);
  if (r) return r;
  // intermediate rows padded to 64 elements: every row starts 256-byte aligned
  const int64_t ldt = (oc + 63) / 64 * 64;
  const size_t img = (size_t)rows * (size_t)ldt * s;
  const bool big = w_rows > mm::cols_max_window(dtype);
  const size_t scr = big ? (size_t)mm::cols_scratch_elems(rows, oc, w_rows) * s : 0;
  if ((r = ensure_tmp(ws, 2 * img + scr))) return r;
  void* tmax = d_max ? ws->tmp : nullptr;  // a null output skips its image
  void* tmin = d_min ? (char*)ws->tmp + img : nullptr;
  void* gscr = big ? (void*)((char*)ws->tmp + 2 * img) : nullptr;
  // row pass: every row is a series of `cols` inputs with window w_cols
  JobArgs a;
  a.mode = 2;
  a.in = d_in;
  a.ld_in = ld_in;
  a.n = cols;
  a.w = w_cols;
  a.omax = tmax;
  a.omin = tmin;
  a.ld_out = ldt;
  const int strat = plan_strategy(dtype, cols, w_cols);
  hipError_t e;
  if (strat == MAXMIN_STRATEGY_TILE) {
    a.run = (int64_t)tuning(dtype).rows_run * mm::kTileOut;
    a.tpr = mm::run_count(cols, w_cols, a.run);
    a.ntiles = a.tpr * rows;
    const int ks = tile_kind(w_cols);
    e = mm::launch_1d(dtype, ks, a, (int)std::min<int64_t>(a.ntiles, mm::grid_cap(dtype, ks)), st);
  } else if (strat == MAXMIN_STRATEGY_RUN) {
    a.run = mm::crun_chunks(cols, w_cols);  // one run per row
    a.tpr = 1;
    a.ntiles = rows;
    e = mm::launch_1d(dtype, mm::kStratRun, a, (int)std::min<int64_t>(a.ntiles, mm::grid_cap(dtype, mm::kStratRun)), st);
  } else {
    a.tpr = mm::chunk_count(cols, w_cols);
    a.ntiles = a.tpr * rows;
    if ((r = ensure_ring(ws, a.ntiles))) return r;
    a.ring = ws->ring;
    a.ring_lg = ws->ring_lg;
    a.ctl = ws->ctl;
    e = mm::launch_1d(dtype, mm::kStratChunk, a, (int)std::min<int64_t>(a.ntiles, mm::grid_cap(dtype, mm::kStratChunk)), st);
  }
  if (e != hipSuccess) return hip_fail(e, "maxmin_filter_2d (rows)");
  // column pass
  const int cp = cols_pass_2d(dtype, w_rows);
  const char* ecb = getenv("MAXMIN_COLS_BAND");
  e = hipErrorNotSupported;
  if (cp == 2)
    e = mm::launch_cols_ring(dtype, tmax, tmin, ldt, rows, oc, w_rows, d_max, d_min, ld_out, ecb ? atoll(ecb) : 0,
                             st);
  if (cp == 1 || (cp == 2 && e == hipErrorNotSupported && w_rows < 16))
    e = mm::launch_f2d_cols(dtype, tmax, tmin, ldt, rows, oc, w_rows, d_max, d_min, ld_out, 0, st);
  if (e == hipErrorNotSupported)
    e = mm::launch_cols(dtype, tmax, tmin, ldt, rows, oc, w_rows, d_max, d_min, ld_out, gscr, st);
  if (e != hipSuccess) return hip_fail(e, "maxmin_filter_2d (columns)");
  return ok();
}

// Centered envelope: the interior is the valid filter of width 2r+1 written
// at offset r; the two truncated ends come from k_env_ends.
int maxmin_envelope(int dtype, const void* d_in, int64_t n, int64_t r, void* d_upper, void* d_lower, void* stream) {
  const size_t s = dsize(dtype);
  if (!s) return fail(MAXMIN_EINVAL, "maxmin_envelope: unknown dtype %d", dtype);
  if (r < 0) return fail(MAXMIN_EINVAL, "maxmin_envelope: radius r=%lld < 0", (long long)r);
  if (n < 0) return fail(MAXMIN_EINVAL, "maxmin_envelope: n=%lld < 0", (long long)n);
  if (n == 0) return ok();
  if (!d_in || !d_upper || !d_lower) return fail(MAXMIN_EINVAL, "maxmin_envelope: null pointer");
  if (!aligned(d_in, s) || !aligned(d_upper, s) || !aligned(d_lower, s))
    return fail(MAXMIN_EINVAL, "maxmin_envelope: pointer not aligned to the element size");
  if (r > (n - 1) / 2 + n) r = (n - 1) / 2 + n;  // larger radii change nothing (and 2r+1 cannot overflow)
  hipStream_t st = (hipStream_t)stream;
  if (n >= 2 * r + 1) {
    JobArgs a;
    a.mode = 0;
    a.a = d_in;
    a.na = n;
    a.n = n;
    a.w = 2 * r + 1;
    a.omax = (char*)d_upper + (size_t)r * s;
    a.omin = (char*)d_lower + (size_t)r * s;
    const int rr = run_series(dtype, a, st, "maxmin_envelope (interior)");
    if (rr) return rr;
  }
  hipError_t e = mm::launch_env_ends(dtype, d_in, n, r, d_upper, d_lower, st);
  if (e != hipSuccess) return hip_fail(e, "maxmin_envelope (ends)");
  return ok();
}

int maxmin_envelope_batched(int dtype, const void* d_in, const int64_t* d_in_offsets, const int64_t* d_radii, int64_t S,
                            void* d_upper, void* d_lower, void* stream) {
  const size_t s = dsize(dtype);
  if (!s) return fail(MAXMIN_EINVAL, "maxmin_envelope_batched: unknown dtype %d", dtype);
  if (S < 0) return fail(MAXMIN_EINVAL, "maxmin_envelope_batched: S < 0");
  if (S == 0) return ok();
  if (!d_in || !d_in_offsets || !d_radii || !d_upper || !d_lower)
    return fail(MAXMIN_EINVAL, "maxmin_envelope_batched: null pointer");
  if (!aligned(d_in, s) || !aligned(d_upper, s) || !aligned(d_lower, s))
    return fail(MAXMIN_EINVAL, "maxmin_envelope_batched: pointer not aligned to the element size");
  hipStream_t st = (hipStream_t)stream;
  Workspace* ws = nullptr;
  int r = get_ws(st, &ws);
  if (r) return r;
  if ((r = ensure_buf(ws, &ws->env, &ws->env_bytes, (size_t)(2 * S + 1) * sizeof(int64_t)))) return r;
  int64_t* wins = (int64_t*)ws->env;
  int64_t* oo = wins + S;
  hipError_t e = mm::launch_env_batched(dtype, d_in, d_in_offsets, d_radii, S, wins, oo, true, nullptr, nullptr, st);
  if (e != hipSuccess) return hip_fail(e, "maxmin_envelope_batched (setup)");
  if ((r = maxmin_filter_batched(dtype, d_in, d_in_offsets, wins, oo, S, d_upper, d_lower, stream))) return r;
  e = mm::launch_env_batched(dtype, d_in, d_in_offsets, d_radii, S, nullptr, nullptr, false, d_upper, d_lower, st);
  if (e != hipSuccess) return hip_fail(e, "maxmin_envelope_batched (ends)");
  return ok();
}

// Grey-scale morphology with a w_rows x w_cols rectangle: erosion is the
// 2-D min filter, dilation the max filter, opening = dilation(erosion),
// closing = erosion(dilation); valid windows throughout.
int maxmin_morph_2d(int dtype, const void* d_in, int64_t rows, int64_t cols, int64_t ld_in, int64_t w_rows,
                    int64_t w_cols, int op, void* d_out, int64_t ld_out, void* stream) {
  const size_t s = dsize(dtype);
  if (!s) return fail(MAXMIN_EINVAL, "maxmin_morph_2d: unknown dtype %d", dtype);
  if (op < MAXMIN_ERODE || op > MAXMIN_CLOSE) return fail(MAXMIN_EINVAL, "maxmin_morph_2d: unknown op %d", op);
  if (w_rows < 1 || w_cols < 1) return fail(MAXMIN_EINVAL, "maxmin_morph_2d: window < 1");
  if (rows < 0 || cols < 0) return fail(MAXMIN_EINVAL, "maxmin_morph_2d: negative size");
  if (ld_in < cols) return fail(MAXMIN_EINVAL, "maxmin_morph_2d: ld_in < cols");
  if (op == MAXMIN_ERODE || op == MAXMIN_DILATE)
    return maxmin_filter_2d(dtype, d_in, rows, cols, ld_in, w_rows, w_cols, op == MAXMIN_DILATE ? d_out : nullptr,
                            op == MAXMIN_ERODE ? d_out : nullptr, ld_out, stream);
  const int64_t r1 = rows - w_rows + 1, c1 = cols - w_cols + 1;
  if (r1 - w_rows + 1 <= 0 || c1 - w_cols + 1 <= 0) return ok();  // no output
  if (ld_out < c1 - w_cols + 1) return fail(MAXMIN_EINVAL, "maxmin_morph_2d: ld_out < output width");
  if (!d_in || !d_out) return fail(MAXMIN_EINVAL, "maxmin_morph_2d: null pointer");
  if (!aligned(d_in, s) || !aligned(d_out, s))
    return fail(MAXMIN_EINVAL, "maxmin_morph_2d: pointer not aligned to the element size");
  hipStream_t st = (hipStream_t)stream;
  Workspace* ws = nullptr;
  int r = get_ws(st, &ws);
  if (r) return r;
  if ((r = ensure_tmp2(ws, (size_t)r1 * (size_t)c1 * s))) return r;
  void* mid = ws->tmp2;
  const bool open = op == MAXMIN_OPEN;  // opening: min first, then max
  if ((r = maxmin_filter_2d(dtype, d_in, rows, cols, ld_in, w_rows, w_cols, open ? nullptr : mid, open ? mid : nullptr,
                            c1, stream)))
    return r;
  return maxmin_filter_2d(dtype, mid, r1, c1, c1, w_rows, w_cols, open ? d_out : nullptr, open ? nullptr : d_out,
                          ld_out, stream);
}

// Autotuner: measure the planner's launch parameters (Tuning) on this
// device for `dtype`, one knob at a time with the others at their best so
// far; a candidate replaces the current value only if it is more than 3%
// faster (run-to-run noise must not move the table).  Inputs are a
// pseudo-random pattern written on the device (selection time does not
// depend on the values).  Each candidate is the best of five timed calls
// after one warm-up.
//  * one series of n elements (0: 2^28): the run length of the tile kernel
//    for w <= 2048 (measured at w = 256) and for 2048 < w <= 8192 (4096);
//    ticket ranges of one-chunk windows (only when the chunk strategy is
//    forced); the long-window strategy (65536); the look-back kernel's
//    ticket ranges (16384, a window that takes it);
//  * the 2-D row pass run length (the series as an image of 8192 columns,
//    63 x 63 windows);
//  * batched calls: per size class with windows up to 8192 (window class x
//    length class), tile or chunk kernel, each measured on a batch of its
//    class (about 2^25 elements); then the tile size (1, 2 or 4 sub-tiles)
//    on a batch shaped like the benchmark's: 10,000 series, lengths
//    log-uniform in [1e3, 1e6], windows uniform in [2, 1024] (fewer series
//    when device memory is short).
int maxmin_autotune(int dtype, int64_t n, void* stream) {
  const size_t s = dsize(dtype);
  if (!s) return fail(MAXMIN_EINVAL, "maxmin_autotune: unknown dtype %d", dtype);
  if (n == 0) n = int64_t(1) << 28;
  if (n < (int64_t(1) << 20)) return fail(MAXMIN_EINVAL, "maxmin_autotune: n=%lld < 2^20", (long long)n);
  hipStream_t st = (hipStream_t)stream;
  if (capturing(st)) return fail(MAXMIN_EBUSY, "maxmin_autotune: the stream is being captured");
  // batches: host descriptions first (sizes decide the buffers)
  struct HostBatch {
    std::vector<int64_t> off, win, oo;
  };
  uint64_t rs = 0x9E3779B97F4A7C15ull;
  auto rnd = [&]() {  // xorshift64*, uniform in [0, 1)
    rs ^= rs >> 12;
    rs ^= rs << 25;
    rs ^= rs >> 27;
    return (double)((rs * 0x2545F4914F6CDD1Dull) >> 11) * (1.0 / 9007199254740992.0);
  };
  auto make = [&](int64_t S, double nlo, double nhi, int64_t wlo, int64_t whi) {
    HostBatch b;
    b.off.assign((size_t)S + 1, 0);
    b.win.resize((size_t)S);
    for (int64_t k = 0; k < S; ++k) {
      const int64_t len = (int64_t)std::floor(std::exp(std::log(nlo) + rnd() * (std::log(nhi) - std::log(nlo))));
      b.off[k + 1] = b.off[k] + len;
      b.win[k] = wlo + (int64_t)(rnd() * (double)(whi - wlo + 1));
      if (b.win[k] > whi) b.win[k] = whi;
    }
    b.oo.assign((size_t)S + 1, 0);
    maxmin_out_offsets(b.off.data(), b.win.data(), S, b.oo.data());
    return b;
  };
  static const double kNLo[3] = {8192.0, 65536.0, 1048576.0}, kNHi[3] = {65535.0, 1048575.0, 4194304.0};
  static const int64_t kWLo[3] = {2, 2049, 4097}, kWHi[3] = {2048, 4096, 8192};
  std::vector<HostBatch> cls;
  for (int wc = 0; wc < 3; ++wc)
    for (int nc = 0; nc < 3; ++nc) {
      const double mean = (kNHi[nc] - kNLo[nc]) / std::log(kNHi[nc] / kNLo[nc]);
      cls.push_back(make(std::max<int64_t>(4, (int64_t)((double)(1 << 25) / mean)), kNLo[nc], kNHi[nc], kWLo[wc],
                         kWHi[wc]));
    }
  size_t fb = 0, tb = 0;
  hipMemGetInfo(&fb, &tb);
  int64_t S4 = 10000;
  while (S4 > 100 && (double)S4 * 144.6e3 * 3.0 * (double)s > 0.4 * (double)fb) S4 /= 2;
  HostBatch big = make(S4, 1e3, 1e6, 2, 1024);
  int64_t maxN = n, maxO = n, maxS = S4;
  for (auto* b : {&big}) {
    maxN = std::max(maxN, b->off.back());
    maxO = std::max(maxO, b->oo.back());
  }
  for (auto& b : cls) {
    maxN = std::max(maxN, b.off.back());
    maxO = std::max(maxO, b.oo.back());
    maxS = std::max<int64_t>(maxS, (int64_t)b.win.size());
  }
  void *in = nullptr, *mx = nullptr, *mn = nullptr;
  int64_t *d_off = nullptr, *d_w = nullptr, *d_oo = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  const Tuning before = tuning(dtype);
  int r = MAXMIN_OK;
  auto cleanup = [&]() {
    if (st) hipStreamSynchronize(st);
    else hipDeviceSynchronize();
    for (void* q : {in, mx, mn, (void*)d_off, (void*)d_w, (void*)d_oo})
      if (q) hipFree(q);
    if (e0) hipEventDestroy(e0);
    if (e1) hipEventDestroy(e1);
  };
  if (hipMalloc(&in, (size_t)maxN * s) != hipSuccess || hipMalloc(&mx, (size_t)maxO * s) != hipSuccess ||
      hipMalloc(&mn, (size_t)maxO * s) != hipSuccess || hipMalloc((void**)&d_off, (maxS + 1) * 8) != hipSuccess ||
      hipMalloc((void**)&d_w, maxS * 8) != hipSuccess || hipMalloc((void**)&d_oo, (maxS + 1) * 8) != hipSuccess) {
    cleanup();
    return fail(MAXMIN_ENOMEM, "maxmin_autotune: cannot allocate its buffers (%lld elements)", (long long)maxN);
  }
  hipError_t e = mm::launch_tune_fill(dtype, in, maxN, st);
  if (e == hipSuccess) e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  if (e != hipSuccess) {
    cleanup();
    return hip_fail(e, "maxmin_autotune");
  }
  auto set = [&](const Tuning& t) {
    std::lock_guard<std::mutex> g(g_tune_mu);
    g_tune[dtype] = t;
    ++g_tune_version;
  };
  auto time_ms = [&](const std::function<int()>& launch) -> float {
    if ((r = launch())) return 0.f;
    float best = 1e30f;
    for (int k = 0; k < 5; ++k) {
      hipEventRecord(e0, st);
      if ((r = launch())) return 0.f;
      hipEventRecord(e1, st);
      hipEventSynchronize(e1);
      float ms = 0.f;
      hipEventElapsedTime(&ms, e0, e1);
      best = std::min(best, ms);
    }
    return best;
  };
  Tuning best = before;
  // try each candidate value of one knob (get / put read and write it)
  auto pick_knob = [&](const std::function<int(const Tuning&)>& get, const std::function<void(Tuning&, int)>& put,
                       std::initializer_list<int> cands, const std::function<int()>& launch) {
    const int cur = get(best);
    float bt = time_ms(launch);
    if (r) return;
    int bv = cur;
    for (int v : cands) {
      if (v == cur) continue;
      Tuning t = best;
      put(t, v);
      set(t);
      const float ms = time_ms(launch);
      if (r) return;
      if (ms < 0.97f * bt) {
        bt = ms;
        bv = v;
      }
    }
    put(best, bv);
    set(best);
  };
  auto pick = [&](int Tuning::*field, std::initializer_list<int> cands, const std::function<int()>& launch) {
    pick_knob([field](const Tuning& t) { return t.*field; }, [field](Tuning& t, int v) { t.*field = v; }, cands,
              launch);
  };
  auto filt = [&](int64_t w) {
    return std::function<int()>([=]() { return maxmin_filter(dtype, in, n, w, mx, mn, stream); });
  };
  pick(&Tuning::tile_run, {2, 4, 8, 16, 32}, filt(256));
  if (!r) pick(&Tuning::tile_run_long, {16, 32, 64, 128}, filt(4096));
  // one-chunk windows run the tile kernel unless the chunk strategy is
  // forced: only then are their ticket ranges worth measuring
  if (!r && plan_strategy(dtype, n, 4096) == MAXMIN_STRATEGY_CHUNK)
    pick(&Tuning::ranges_one, {0, 8, 16, 32}, filt(4096));
  if (!r && n >= 4 * 65536) pick(&Tuning::long_strategy, {MAXMIN_STRATEGY_CHUNK, MAXMIN_STRATEGY_RUN}, filt(65536));
  if (!r && n >= 4 * 16384 && best.long_strategy == MAXMIN_STRATEGY_CHUNK && long_lookback(16384))
    pick(&Tuning::ranges_long, {0, 16}, filt(16384));
  if (!r)  // the series as an image of 8192 columns, 63 x 63 windows (rows then columns)
    pick(&Tuning::rows_run, {8, 16, 32}, std::function<int()>([=]() {
           const int64_t cols = 8192, rows = n / cols;
           return maxmin_filter_2d(dtype, in, rows, cols, cols, 63, 63, mx, mn, cols - 62, stream);
         }));
  // batched: a batch's descriptors go to the device, then its call is timed
  auto upload = [&](const HostBatch& b) -> std::function<int()> {
    const int64_t S = (int64_t)b.win.size();
    hipError_t ee = hipMemcpyAsync(d_off, b.off.data(), (S + 1) * 8, hipMemcpyHostToDevice, st);
    if (ee == hipSuccess) ee = hipMemcpyAsync(d_w, b.win.data(), S * 8, hipMemcpyHostToDevice, st);
    if (ee == hipSuccess) ee = hipMemcpyAsync(d_oo, b.oo.data(), (S + 1) * 8, hipMemcpyHostToDevice, st);
    if (ee == hipSuccess) ee = st ? hipStreamSynchronize(st) : hipDeviceSynchronize();
    if (ee != hipSuccess) r = hip_fail(ee, "maxmin_autotune (batch descriptors)");
    return [=]() { return maxmin_filter_batched(dtype, in, d_off, d_w, d_oo, S, mx, mn, stream); };
  };
  for (int wc = 0; wc < 3 && !r; ++wc)
    for (int nc = 0; nc < 3 && !r; ++nc) {
      auto launch = upload(cls[wc * 3 + nc]);
      if (r) break;
      pick_knob([wc, nc](const Tuning& t) { return (int)t.batch.strat[wc][nc]; },
                [wc, nc](Tuning& t, int v) { t.batch.strat[wc][nc] = (uint8_t)v; }, {mm::kBatchTile, mm::kBatchChunk},
                launch);
    }
  if (!r) {
    auto launch = upload(big);
    if (!r)
      pick_knob([](const Tuning& t) { return (int)t.batch.run_subtiles; },
                [](Tuning& t, int v) { t.batch.run_subtiles = v; }, {1, 2, 4}, launch);
  }
  const int rr = r;
  cleanup();
  if (rr) {
    set(before);
    return rr;
  }
  best.tuned = 1;
  set(best);
  {
    // graphs captured for the temporary buffers are of no further use
    Workspace* ws = nullptr;
    if (get_ws(st, &ws) == MAXMIN_OK) drop_graphs(ws);
  }
  return ok();
}

// The current table for `dtype` (MAXMIN_TUNING_LEN entries).
int maxmin_tuning(int dtype, int64_t* out) {
  if (!dsize(dtype)) return fail(MAXMIN_EINVAL, "maxmin_tuning: unknown dtype %d", dtype);
  if (!out) return fail(MAXMIN_EINVAL, "maxmin_tuning: null pointer");
  const Tuning t = tuning(dtype);
  out[0] = t.tile_run;
  out[1] = t.tile_run_long;
  out[2] = t.rows_run;
  out[3] = t.ranges_one;
  out[4] = t.ranges_long;
  out[5] = t.long_strategy;
  out[6] = t.batch.run_subtiles;
  for (int wc = 0; wc < 3; ++wc)
    for (int nc = 0; nc < 3; ++nc) out[7 + wc * 3 + nc] = t.batch.strat[wc][nc];
  out[16] = t.tuned;
  return ok();
}

// Synchronise `stream` and report whether any look-back wait on it gave up.
int maxmin_check_stream(void* stream) {
  hipStream_t st = (hipStream_t)stream;
  hipError_t e = st ? hipStreamSynchronize(st) : hipDeviceSynchronize();
  if (e != hipSuccess) return hip_fail(e, "maxmin_check_stream");
  int dev = 0;
  hipGetDevice(&dev);
  Workspace* ws = nullptr;
  {
    std::lock_guard<std::mutex> g(g_mu);
    auto it = g_ws.find(std::make_pair(dev, st));
    if (it == g_ws.end()) return ok();
    ws = it->second;
  }
  mm::Ctl c;
  e = hipMemcpy(&c, ws->ctl, sizeof c, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(e, "maxmin_check_stream (read)");
  if (c.err) return fail(MAXMIN_EDEVICE, "a look-back wait on this stream timed out (results invalid)");
  return ok();
}

}  // extern "C"
