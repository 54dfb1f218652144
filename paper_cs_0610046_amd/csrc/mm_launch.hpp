// Host-side launchers of the gfx950 kernels (internal to libmaxmin).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mm_device.hpp"

namespace mm {

// Tile strategy: a workgroup streams through runs of consecutive windows in
// sub-tiles of kTileOut positions.
constexpr int kTileThreads = 256;
constexpr int kTileV = 8;                                   // positions per thread
constexpr int kTileOut = kTileThreads * kTileV;             // 2048 positions per sub-tile
constexpr int kTileMaxBlock = kTileV * 128;                 // largest block: 128 lanes, two wavefronts
constexpr int64_t kTileMaxW = 2 * kTileMaxBlock;            // 2048: w <= 2 * block size, w - 1 <= sub-tile
// Second instantiation (kStratTile2, single series and rows): blocks of a
// whole sub-tile, windows end at most two sub-tiles after they start.
constexpr int64_t kTileMaxW2 = 2 * kTileOut;                // 4096
// ... and with windows ending three or four sub-tiles on (kStratTile3/4)
constexpr int64_t kTileMaxW4 = 4 * kTileOut;                // 8192
// Longest run: on MI355X (n = 2^28 and 2^30 float32) runs of 16 sub-tiles,
// dealt round robin, beat one long run per workgroup by 5-6%.
constexpr int64_t kTileRunMax = 16 * kTileOut;
// Tile of a described-series job (batched calls, serving batches): one
// sub-tile of windows; each workgroup streams a contiguous range of tiles.
constexpr int64_t kRunBatched = kTileOut;

// Chunk strategy: window-aligned chunks of at most kChunkMax inputs.
constexpr int kChunkThreads = 256;
constexpr int kChunkV = 16;
constexpr int kChunkMax = kChunkThreads * kChunkV;          // 4096

// Chunk runs: window-aligned chunks of at most kCrMax inputs, aggregates in
// an LDS ring of kCrRing chunks (so K = ceil(w / kCrMax) <= kCrRing).
constexpr int kCrV = 8;
constexpr int kCrMax = kChunkThreads * kCrV;                // 2048
constexpr int kCrRing = 1024;

__host__ __device__ inline int64_t crun_chunks(int64_t n, int64_t w) {
  if (n < w || n <= 0) return 0;
  int64_t K = (w + kCrMax - 1) / kCrMax;
  int64_t C = (w + K - 1) / K;
  int64_t last = n - 1;
  return (last / w) * K + (last % w) / C + 1;
}

// Batched calls: every series falls in a size class by its window (w <=
// 2048, <= 4096, <= 8192, longer) and its length (n < 2^16, < 2^20,
// longer); a plan gives each class a strategy: the tile kernel of the lag
// that fits the window (classes up to 8192) or the chunk kernel.  The
// series of one path share a launch: kBatchNP tile-prefix arrays, one per
// path (tile lag 1..4, chunk).
constexpr int kBatchWClasses = 4, kBatchNClasses = 3, kBatchNP = 5;
constexpr int kBatchChunkPath = 4;
enum BatchStrategy : uint8_t { kBatchTile = 0, kBatchChunk = 1 };
struct BatchPlan {
  uint8_t strat[kBatchWClasses][kBatchNClasses];  // BatchStrategy per class
  int32_t run_subtiles;                             // tile of the tile paths, in sub-tiles
};
__host__ __device__ inline int batch_wclass(int64_t w) {
  return w <= 2048 ? 0 : (w <= 4096 ? 1 : (w <= 8192 ? 2 : 3));
}
__host__ __device__ inline int batch_nclass(int64_t n) { return n < (1 << 16) ? 0 : (n < (1 << 20) ? 1 : 2); }
// Which launch serves a series: 0..3 the tile kernel of lag 1..4, 4 the
// chunk kernel; -1 when the series has no complete window.
__host__ __device__ inline int batch_path(const BatchPlan& p, int64_t n, int64_t w) {
  if (w < 1 || n < w) return -1;
  const int wc = batch_wclass(w);
  if (wc == 3 || p.strat[wc][batch_nclass(n)] == kBatchChunk) return kBatchChunkPath;
  return w <= 2048 ? 0 : (int)((w - 1) / 2048);  // lag 1; 2 (<= 4096); 3 (<= 6144); 4 (<= 8192)
}
// Tiles of a series on its path: runs of `run` windows, or chunks.
__host__ __device__ inline int64_t batch_tiles(int path, int64_t n, int64_t w, int64_t run);

// Batched envelopes: a series of at most kEnvShortN samples with radius at
// most kEnvShortR is served whole by one wavefront (k_env_short); the others
// by the batched filter plus the end scans.  Decided on the device.
constexpr int64_t kEnvShortN = 16384;
constexpr int64_t kEnvShortR = 256;  // window 2r+1 <= 513 = one 512-position segment + 1
__host__ __device__ inline bool env_short(int64_t n, int64_t r) {
  return n > 0 && n <= kEnvShortN && r >= 0 && r <= kEnvShortR;
}

// Runs of `run` windows covering the n - w + 1 windows of a series.
__host__ __device__ inline int64_t run_count(int64_t n, int64_t w, int64_t run) {
  int64_t no = n - w + 1;
  return no > 0 ? (no + run - 1) / run : 0;
}
// Run length for a single series on `grid` workgroups: about one run per
// workgroup, a multiple of the sub-tile, at most `cap` (kTileRunMax unless
// the autotuner chose another).
inline int64_t run_length(int64_t nout, int64_t grid, int64_t cap = kTileRunMax) {
  int64_t r = (nout + grid - 1) / grid;
  r = (r + kTileOut - 1) / kTileOut * kTileOut;
  r = r < kTileOut ? kTileOut : r;
  return r > cap ? cap : r;
}
// Number of chunk tiles covering [0, n) for window w (0 if n < w: no output),
// chunks of at most cmax inputs.
__host__ __device__ inline int64_t chunk_count(int64_t n, int64_t w, int64_t cmax = kChunkMax) {
  if (n < w || n <= 0) return 0;
  int64_t K = (w + cmax - 1) / cmax;
  int64_t C = (w + K - 1) / K;
  int64_t last = n - 1;
  return (last / w) * K + (last % w) / C + 1;
}
// Chunk size of the two-pass long-window kernels: chunks of at most 2048
// (eight positions per thread, five workgroups per CU instead of three)
// where that measured faster on MI355X (n = 2^28 float32), else of 4096:
// up to w = 65536 for blocks of whole 4096-element chunks or of at most
// three chunks.  2048 / 4096: w = 9000 1.06 / 1.07 ms, 10000 1.00 / 1.24,
// 65536 0.94 / 0.97, but 40000 0.98 / 0.94, 262144 0.99 / 0.86 and 2^20
// 1.17 / 0.94.
constexpr int kColVShort = 8;
int long_col_v_override();  // MAXMIN_LONG_V = 8 / 16 (experiments), else 0
inline int long_col_v(int64_t w) {
  if (const int v = long_col_v_override()) return v;
  const int64_t K = (w + kChunkMax - 1) / kChunkMax;
  const bool whole = K * kChunkMax == w;
  return w <= 65536 && (whole || K <= 3) ? kColVShort : kChunkV;
}
inline int64_t long_chunk_max(int64_t w) { return int64_t(kChunkThreads) * long_col_v(w); }
// The one-pass kernel (k_chunk_col1): chunks of 2048 only while a window
// spans at most three 4096-element chunks.  On MI355X (n = 2^28 float32),
// 2048 / 4096: w = 8193 1.17 / 1.20 ms, 10000 0.88 / 1.04, 20000 0.88 /
// 0.77, 65536 0.87 / 0.77, 131072 0.91 / 0.78, 2^20 1.26 / 0.89.
// 8-byte data always takes chunks of 2048 (16 KiB, as 4096 of 4-byte data;
// 4096 of them need 268 VGPRs: one workgroup per CU).
inline int long1_col_v(int64_t w, size_t elem) {
  if (const int v = long_col_v_override()) return v;
  return elem == 8 || (w + kChunkMax - 1) / kChunkMax <= 3 ? kColVShort : kChunkV;
}

__host__ __device__ inline int64_t batch_tiles(int path, int64_t n, int64_t w, int64_t run) {
  if (path < 0) return 0;
  return path == kBatchChunkPath ? chunk_count(n, w) : run_count(n, w, run);
}

// Type-erased description of a 1-D launch (converted to Job<T> inside).
struct JobArgs {
  int mode = 0;  // 0 single series, 1 described series, 2 rows
  // single series: element i is a[i] (i < na) else b[i - na]
  const void* a = nullptr;
  const void* b = nullptr;
  int64_t na = 0;
  int64_t n = 0;  // also the row length in mode 2
  int64_t w = 0;
  void* omax = nullptr;
  void* omin = nullptr;
  void* carry = nullptr;
  int64_t ntiles = 0;
  // described series
  const void* descs = nullptr;
  const int64_t* pre = nullptr;
  int64_t S = 0;
  // rows
  const void* in = nullptr;
  int64_t ld_in = 0;
  int64_t ld_out = 0;
  int64_t tpr = 0;
  int64_t run = 0;  // tile strategy: windows per run
  int64_t* amax = nullptr;  // arg filter outputs (single series, tile strategy only)
  int64_t* amin = nullptr;
  int ranges = 0;   // chunk strategy, single series: ticket ranges (0 or 1: one counter)
  // chunk strategy look-back state
  uint64_t* ring = nullptr;
  uint32_t ring_lg = 0;
  Ctl* ctl = nullptr;
};

// kStratArg: the tile kernel carrying locations (arg max/min filter).
// kStratTile2 / kStratArg2: the same kernels for 2048 < w <= 4096 (single
// series, rows); kStratTile3 / kStratTile4: 4096 < w <= 6144 / 6144 < w <=
// 8192.
enum Strategy : int {
  kStratTile = 1,
  kStratChunk = 2,
  kStratRun = 3,
  kStratArg = 4,
  kStratTile2 = 5,
  kStratArg2 = 6,
  kStratTile3 = 7,
  kStratTile4 = 8
};

// Occupancy-derived persistent grid sizes (computed once per device).
int grid_cap(int dtype, int strategy);

hipError_t launch_1d(int dtype, int strategy, const JobArgs& a, int grid, hipStream_t st);
// One series (a.mode 0, w <= kTileMaxW4) with the tile kernel: run length
// and grid as the planner sets them (mm_abi.cpp); no scratch memory.
hipError_t launch_tile_series(int dtype, JobArgs a, hipStream_t st);
// Single series (a.mode 0) with more than one chunk per block of w: chunk
// aggregates into agg (2 * chunk_count(n, w, long_chunk_max(w)) elements),
// then one column of chunks per workgroup (no look-back, no re-read of the
// chunk w back).
hipError_t launch_long(int dtype, const JobArgs& a, void* agg, hipStream_t st);
// The same in one pass (no aggregate pass): each column workgroup publishes
// its chunk's max and min as tagged records in rec (4 words per chunk,
// long1_records(n, w) chunks) and reads its siblings'; needs the stream's
// control words (epoch) and a cooperative launch (hipErrorNotSupported when
// a column group does not fit on the device).
int64_t long1_records(int dtype, int64_t n, int64_t w);
hipError_t launch_long1(int dtype, const JobArgs& a, uint64_t* rec, Ctl* ctl, hipStream_t st);

// Batched setup: fills S descriptors (bytes: S * series_bytes()) and the
// kBatchNP per-path tile prefix sums pre + p (S + 1), p = 0..kBatchNP-1
// (batch_pre_len(S) entries in all, the per-workgroup totals included).
constexpr int64_t kBatchMaxGroups = 1024;
inline int64_t batch_pre_len(int64_t S) { return kBatchNP * (S + 1) + kBatchNP * (kBatchMaxGroups + 1); }
hipError_t launch_batched_setup(int dtype, const void* d_in, const int64_t* in_off, const int64_t* wins,
                                const int64_t* out_off, int64_t S, void* d_max, void* d_min, void* descs,
                                int64_t* pre, const BatchPlan& plan, hipStream_t st);

// Serving batches: many small host <-> device copies in one launch.  Each
// piece copies `bytes` from src to dst (device addresses; host buffers must
// be pinned and mapped, which hipHostMalloc memory is), one workgroup at a
// time each.  A workgroup keeps 16 KiB of host reads in flight, so buffers
// are cut into pieces of that size to spread them over workgroups.
struct CopyPiece {
  const char* src;
  char* dst;
  int64_t bytes;
};
constexpr int64_t kCopyPieceMax = int64_t(16) << 10;
hipError_t launch_copy_pieces(const CopyPiece* pieces, int64_t np, hipStream_t st);

// The autotuner's input: n elements of a pseudo-random pattern.
hipError_t launch_tune_fill(int dtype, void* a, int64_t n, hipStream_t st);
// The batched plan the planner uses for dtype (tuned or default, with the
// experiment overrides), for launches made outside mm_abi.cpp.
BatchPlan batch_plan_for(int dtype);

// A stream push that completes no window: new carry = last min(n, w-1)
// samples of (a[0..na) ++ b).
hipError_t launch_carry_only(int dtype, const JobArgs& a, hipStream_t st);
// Centered envelopes: the two truncated ends of one series; for a batch,
// either the setup of the interiors' window / output-offset arrays (setup)
// or the ends of every series.
hipError_t launch_env_ends(int dtype, const void* a, int64_t n, int64_t r, void* up, void* lo, hipStream_t st);
hipError_t launch_env_batched(int dtype, const void* in, const int64_t* off, const int64_t* radii, int64_t S,
                              int64_t* wins, int64_t* oo, bool setup, void* up, void* lo, hipStream_t st);
// The short series of a batched envelope call (env_short), one wavefront each.
hipError_t launch_env_short(int dtype, const void* in, const int64_t* off, const int64_t* radii, int64_t S, void* up,
                            void* lo, hipStream_t st);
// One step of the arg filter's long-window path (see k_argcombine): window
// p's outputs j < nout from F reads of window q's value/location arrays.
// Long-window arg filter, one step: from the level of window q (values and
// int64 locations, nlv = n - q + 1 entries each) to window w, F = w / q in
// 2..kArgColsMaxF rows of q entries plus, if Fq < w, the entry at j+w-q
// ((F+1)q >= w required).  hipErrorInvalidValue outside those limits.
constexpr int64_t kArgColsMaxF = 31;
// Arg filter for 4096 < w <= 2^29 in two passes over chunks (per-chunk
// leftmost max / min, then columns of chunks): scratch of
// arg_chunk_scratch(dtype, n, w) bytes, 16-byte aligned.
size_t arg_chunk_scratch(int dtype, int64_t n, int64_t w);
hipError_t launch_arg_chunks(int dtype, const void* d_in, int64_t n, int64_t w, void* scratch, void* ox, int64_t* jx,
                             void* on, int64_t* jn, hipStream_t st);
hipError_t launch_arg_cols(int dtype, const void* vx, const int64_t* ix, const void* vn, const int64_t* in,
                           int64_t nlv, int64_t q, int64_t w, int64_t nout, void* ox, int64_t* jx, void* on,
                           int64_t* jn, hipStream_t st);
hipError_t launch_arg_combine(int dtype, const void* vx, const void* vn, const int64_t* ix, const int64_t* in_,
                              int64_t q, int64_t p, int F, int64_t nout, void* ox, void* on, int64_t* jx, int64_t* jn,
                              hipStream_t st);

size_t series_bytes();

// Per-stream look-back state owned by the ABI layer (see mm_abi.cpp).
int stream_lookback_state(hipStream_t stream, int64_t ntiles, uint64_t** ring, uint32_t* lg, Ctl** ctl);
// Record a thread-local error message for maxmin_last_error; returns code.
int set_error(int code, const char* msg);

// 2-D column pass over the row-filtered images (rows x oc, leading
// dimension ld_t): max-filter tmax's columns and min-filter tmin's.
// Windows above cols_max_window(dtype) keep their per-block suffixes in a
// global scratch of cols_scratch_elems(rows, oc, wr) elements (else pass null).
hipError_t launch_cols(int dtype, const void* tmax, const void* tmin, int64_t ld_t, int64_t rows, int64_t oc,
                       int64_t wr, void* d_max, void* d_min, int64_t ld_out, void* gscratch, hipStream_t st);
int64_t cols_max_window(int dtype);
// Column pass streaming down bands of output rows with each column's block
// in an LDS ring (float32 / int32 / uint16; each lane takes 1, 2 or 4
// 32-bit words of a row, so ld_t must be a multiple of the words' elements
// and the images aligned to the access), w_rows <= 64, else
// hipErrorNotSupported.  Either image may be null for a one-output call.
// band_rows <= 0: the launcher picks the band height.
hipError_t launch_cols_ring(int dtype, const void* tmax, const void* tmin, int64_t ld_t, int64_t rows, int64_t oc,
                            int64_t wr, void* d_max, void* d_min, int64_t ld_out, int64_t band_rows,
                            hipStream_t st);

// Fused 2-D filter (one pass, no intermediate images) for w_rows <= 64 and
// w_cols <= 64 * V + 1 (V = 4, 4, 4, 2, 1, 1 for column blocks 1..32);
// hipErrorNotSupported when the windows do not fit.  band_rows <= 0: the
// launcher picks the band height.
bool f2d_eligible(int dtype, int64_t w_rows, int64_t w_cols);
hipError_t launch_f2d(int dtype, const void* d_in, int64_t ld_in, int64_t rows, int64_t cols, int64_t w_rows,
                      int64_t w_cols, void* d_max, void* d_min, int64_t ld_out, int64_t band_rows, hipStream_t st);
// The same kernel's column filter alone, as the second pass of
// rows-then-columns over the row-filtered images (rows x oc, leading
// dimension ld_t; either may be null for a one-output call): w_rows <= 64,
// else hipErrorNotSupported (launch_cols serves those).
hipError_t launch_f2d_cols(int dtype, const void* tmax, const void* tmin, int64_t ld_t, int64_t rows, int64_t oc,
                           int64_t w_rows, void* d_max, void* d_min, int64_t ld_out, int64_t band_rows,
                           hipStream_t st);
int64_t cols_scratch_elems(int64_t rows, int64_t oc, int64_t wr);

}  // namespace mm
