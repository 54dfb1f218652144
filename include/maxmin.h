/*
 * maxmin.h -- C ABI of the MI355X (gfx950) running max-min filter library.
 *
 * The running max-min filter (D. Lemire, "Streaming Maximum-Minimum Filter
 * Using No More than Three Comparisons per Element", Section 1): for a series
 * a_0 .. a_{n-1} and a window width w, compute for every window [j, j+w)
 *     max[j] = max{a_j, ..., a_{j+w-1}},   min[j] = min{a_j, ..., a_{j+w-1}},
 * for j = 0 .. n-w (0-based, valid windows only: n_out = max(0, n-w+1)).
 *
 * Conventions shared by every entry point:
 *   - Pointers named d_* are DEVICE pointers (hipMalloc'd, or torch CUDA
 *     tensors); pointers named h_* are HOST pointers.  The caller owns all of
 *     them; the library never frees or retains them past the call (except
 *     the state a maxmin_stream_t handle owns, see below).
 *   - Device pointers must be aligned to the element size; any such
 *     alignment is accepted.  d_max, d_min and the input must not overlap.
 *   - `stream` is a hipStream_t passed as void* (NULL = the default
 *     stream).  Every call enqueues its work on that stream and returns
 *     without synchronising; results are ready once the stream has reached
 *     the call.  Calls that overlap on different streams are independent
 *     (the library keeps its scratch memory per stream).
 *   - Values are only compared and selected, never combined arithmetically,
 *     so results are bit-exact.  Float inputs must be NaN-free; a window
 *     holding both +0.0 and -0.0 returns one of them unspecified.
 *   - Sizes and offsets are int64.  w > n is not an error: it yields no
 *     output.
 *   - Return value: MAXMIN_OK (0) or a negative maxmin_status_t.  On error
 *     nothing is enqueued and maxmin_last_error() describes the failure
 *     (thread-local).  No entry point throws or aborts.
 */
#ifndef MAXMIN_H
#define MAXMIN_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  MAXMIN_F32 = 0,
  MAXMIN_F64 = 1,
  MAXMIN_I32 = 2, /* signed order */
  MAXMIN_U16 = 3  /* unsigned order */
} maxmin_dtype_t;

typedef enum {
  MAXMIN_OK = 0,
  MAXMIN_EINVAL = -1,      /* bad argument (w < 1, n < 0, null pointer with work to do, bad ld, ...) */
  MAXMIN_ENOMEM = -2,      /* the library could not allocate its scratch memory */
  MAXMIN_EDEVICE = -3,     /* a HIP call failed */
  MAXMIN_EBUSY = -4,       /* scratch memory would have to grow while the stream is being captured */
  MAXMIN_EUNSUPPORTED = -5 /* dtype or size outside what the library supports */
} maxmin_status_t;

/* Strategies a call may use; all produce identical bits. */
typedef enum {
  MAXMIN_STRATEGY_AUTO = 0,  /* planner / autotuner decides */
  MAXMIN_STRATEGY_TILE = 1,  /* LDS tile: power-of-two block prefix/suffix plus whole blocks between (w <= 8192; series of a batched call: w <= 2048) */
  MAXMIN_STRATEGY_CHUNK = 2, /* window-aligned chunks: cross-workgroup look-back over chunk aggregates, or (one series, most windows of several chunks) chunk aggregates first, then columns of chunks (any w) */
  MAXMIN_STRATEGY_RUN = 3    /* window-aligned chunks walked in runs, aggregates kept per workgroup (any w) */
} maxmin_strategy_t;

/*
 * maxmin_filter -- one series (Section 1 definition).
 *   d_in  : n elements of `dtype`, contiguous.
 *   d_max, d_min : n_out = max(0, n-w+1) elements each, contiguous.  One of
 *                  them may be NULL: a max-only or min-only filter (that
 *                  output is neither computed into memory nor stored).
 *                  The same holds for the batched, stream and 2-D calls.
 * Errors: EINVAL if w < 1, n < 0, or d_in (or both outputs) is null while
 * n_out > 0.
 */
int maxmin_filter(int dtype, const void* d_in, int64_t n, int64_t w, void* d_max,
                  void* d_min, void* stream);

/*
 * maxmin_filter_noalloc -- maxmin_filter that allocates nothing, for callers
 * that cannot call hipMalloc: code under HIP graph capture, tight serving
 * loops, harnesses that forbid allocation.  Same arguments, outputs and
 * bits as maxmin_filter; the caller passes the inputs and outputs as usual.
 *   Scratch: windows w <= 8192 need none.  Longer windows keep their chunk
 *   aggregates (2 * chunks * element size bytes, chunks <= n / 1024 + 1) in
 *   a fixed 32 MiB device array inside the library, which every GPU the
 *   library runs on holds until the process ends; a call that would need
 *   more (e.g. more than 2^31 elements of 8-byte data) returns
 *   MAXMIN_EUNSUPPORTED before enqueuing anything.  Nothing in the array
 *   needs clearing (the first pass writes every aggregate the second reads).
 *   Calls with w > 8192 that overlap on one GPU (different streams, or
 *   different host threads) share that array and race: serialise them.
 *   Forced strategies (maxmin_set_strategy) are ignored: w <= 8192 takes the
 *   tile kernel, longer windows the two-pass chunk kernels.
 * Errors: as maxmin_filter, plus EUNSUPPORTED (scratch too small).
 */
int maxmin_filter_noalloc(int dtype, const void* d_in, int64_t n, int64_t w, void* d_max,
                          void* d_min, void* stream);

/*
 * maxmin_argfilter -- one series: the window max and min (as maxmin_filter)
 * and their locations (Section 5: an implementation that stores locations
 * gives the arg max/min filter at no extra cost).  Ties: the LEFTMOST
 * location of the window's max, and of its min.
 *   d_argmax, d_argmin : n_out int64 each, 0-based positions in d_in.
 * w <= 4096 runs the tile kernel with (value, location) pairs; longer
 * windows start from it at a window q <= 4096 and then either take one
 * running window over rows of q level entries (8192 < w <= 31 x 4096) or
 * combine steps (window p as the union of F <= 16 overlapping windows of
 * ceil(p/F)), through library scratch of up to 2 x n x (2 s + 16) bytes,
 * grown outside graph capture (EBUSY inside one).
 * Errors: EINVAL if w < 1, n < 0, or a pointer is null or misaligned while
 * n_out > 0; ENOMEM if the scratch cannot be allocated.
 */
int maxmin_argfilter(int dtype, const void* d_in, int64_t n, int64_t w, void* d_max, void* d_min,
                     int64_t* d_argmax, int64_t* d_argmin, void* stream);

/*
 * maxmin_filter_batched -- S independent series in one packed buffer, each
 * with its own window (Section 1 definition applied per series).
 *   d_in_offsets [S+1] : series k is d_in[d_in_offsets[k] .. d_in_offsets[k+1]),
 *                        non-decreasing, d_in_offsets[0] = 0.
 *   d_windows    [S]   : w_k >= 1.
 *   d_out_offsets[S+1] : series k writes its max(0, n_k-w_k+1) outputs to
 *                        d_max/d_min[d_out_offsets[k] ..]; computed by
 *                        maxmin_out_offsets (host) from the same arrays.
 * All three arrays are DEVICE int64 arrays.  Their contents are not
 * validated on the host (that would need a synchronisation); malformed
 * offsets are undefined behaviour.
 * Errors: EINVAL if S < 0 or a pointer is null while S > 0.
 */
int maxmin_filter_batched(int dtype, const void* d_in, const int64_t* d_in_offsets,
                          const int64_t* d_windows, const int64_t* d_out_offsets,
                          int64_t S, void* d_max, void* d_min, void* stream);

/*
 * maxmin_out_offsets -- host helper: h_out_offsets[0] = 0 and
 * h_out_offsets[k+1] = h_out_offsets[k] + max(0, n_k - w_k + 1), with
 * n_k = h_in_offsets[k+1] - h_in_offsets[k].  All arrays are HOST arrays.
 * Errors: EINVAL on null pointers, decreasing offsets or a window < 1.
 */
int maxmin_out_offsets(const int64_t* h_in_offsets, const int64_t* h_windows, int64_t S,
                       int64_t* h_out_offsets);

/*
 * Streams -- the filter applied to a series that arrives in chunks, with
 * zero stream latency (Section 1's definition of stream latency): each push
 * emits exactly the windows whose last sample is in the chunk, so the
 * concatenation of all pushes' outputs equals maxmin_filter over the
 * concatenated input.  The handle owns a device-resident carry of the last
 * min(t, w-1) samples (t = samples pushed so far, int64) and a host copy
 * of t; nothing else is kept.
 *
 * maxmin_stream_create: allocates the handle and its device carry on the
 *   current device.  Errors: EINVAL (w < 1, bad dtype, null out), ENOMEM.
 * maxmin_stream_push: d_chunk has m elements; d_max/d_min must hold at least
 *   m elements each; *h_n_out receives max(0, t+m-w+1) - max(0, t-w+1),
 *   computed on the host before anything is enqueued.  Pushes on one handle
 *   must be issued in order on one stream (each reads the carry the
 *   previous one wrote).  Errors: EINVAL (null handle, m < 0, null pointers
 *   with work to do).
 * maxmin_stream_destroy: frees the handle and its device carries after
 *   waiting for the handle's last push to finish (an event recorded on that
 *   push's stream; no device-wide synchronisation).  NULL is accepted.
 * maxmin_stream_samples: samples pushed so far (t), or -1 for NULL.
 * maxmin_stream_export: the stream's whole state, (t, its last min(t, w-1)
 *   samples): waits for the handle's last push, copies the samples (oldest
 *   first) into h_carry (host memory, capacity >= min(t, w-1) elements, may
 *   be NULL when that is 0) and t into *h_t.  The handle is unchanged.
 *   Errors: EINVAL (null handle or h_t, null h_carry with samples to copy),
 *   EDEVICE.
 * maxmin_stream_import: a new handle on the current device that continues
 *   from an exported state (dtype and w as the stream was created with):
 *   pushing to it emits exactly what pushing to the original would have
 *   (checkpoint / resume, or moving a stream to another device or process).
 *   The caller keeps h_carry.  Errors: EINVAL (w < 1, t < 0, bad dtype,
 *   null out, null h_carry with samples to copy), ENOMEM, EDEVICE.
 */
typedef struct maxmin_stream maxmin_stream_t;
int maxmin_stream_create(int dtype, int64_t w, maxmin_stream_t** out);
int maxmin_stream_push(maxmin_stream_t* st, const void* d_chunk, int64_t m, void* d_max,
                       void* d_min, int64_t* h_n_out, void* stream);
int maxmin_stream_destroy(maxmin_stream_t* st);
int64_t maxmin_stream_samples(const maxmin_stream_t* st);
int maxmin_stream_export(const maxmin_stream_t* st, void* h_carry, int64_t* h_t);
int maxmin_stream_import(int dtype, int64_t w, int64_t t, const void* h_carry, maxmin_stream_t** out);

/*
 * maxmin_filter_2d -- the 1-D filter applied to rows, then to columns
 * (Section 1, images): for a row-major image with leading dimension ld_in
 * (elements), outputs (rows-w_rows+1) x (cols-w_cols+1) with leading
 * dimension ld_out:
 *   max[r][c] = max over a[r..r+w_rows)[c..c+w_cols),  min likewise.
 * Errors: EINVAL if a window < 1, rows/cols < 0, ld_in < cols,
 * ld_out < output width, or a null pointer with work to do.
 */
int maxmin_filter_2d(int dtype, const void* d_in, int64_t rows, int64_t cols, int64_t ld_in,
                     int64_t w_rows, int64_t w_cols, void* d_max, void* d_min, int64_t ld_out,
                     void* stream);

/*
 * maxmin_envelope -- centered envelope of radius r >= 0 (the precomputed
 * max-min filter used to bound the time warping distance, Section 1):
 *   d_upper[i] = max of d_in over [max(0, i-r), min(n-1, i+r)], d_lower
 *   likewise; n outputs each (windows truncated at the series ends).
 * The interior runs the 1-D filter with w = 2r+1; the two ends are scans.
 * Errors: EINVAL if r < 0, n < 0, or a pointer is null / misaligned while
 * n > 0.
 */
int maxmin_envelope(int dtype, const void* d_in, int64_t n, int64_t r, void* d_upper, void* d_lower,
                    void* stream);

/*
 * maxmin_envelope_batched -- the envelope of each of S packed series, with
 * per-series radii: series k is d_in[d_in_offsets[k] .. d_in_offsets[k+1])
 * with radius d_radii[k] >= 0, and its envelope goes to the same positions
 * of d_upper / d_lower.  d_in_offsets [S+1] and d_radii [S] are DEVICE int64
 * arrays, not validated on the host (a negative radius leaves that series'
 * outputs unwritten).  Uses library scratch of (2S+1) int64 and the batched
 * filter (graph replay on repeat).
 * Errors: EINVAL if S < 0 or a pointer is null while S > 0.
 */
int maxmin_envelope_batched(int dtype, const void* d_in, const int64_t* d_in_offsets,
                            const int64_t* d_radii, int64_t S, void* d_upper, void* d_lower,
                            void* stream);

/*
 * maxmin_autotune -- measure the planner's launch parameters for `dtype` on
 * the current device and keep the fastest, process-wide (a value changes
 * only when more than 3% faster): the tile kernel's run length for w <=
 * 2048 and for 2048 < w <= 8192, the ticket-range counts of the look-back
 * chunk kernel, the strategy for w > 8192 (chunk or chunk runs), the run
 * length of the 2-D row pass, and the batched plan: for every size class
 * with windows up to 8192 -- window class (<= 2048, <= 4096, <= 8192) by
 * length class (n < 2^16, < 2^20, longer) -- the tile or the chunk kernel,
 * each measured on a batch of that class, then the batched tile size (1, 2
 * or 4 sub-tiles of 2048 windows) on a batch shaped like 10,000 series of
 * lengths log-uniform in [1e3, 1e6] with windows in [2, 1024] (fewer series
 * if device memory is short).  Single-series knobs are measured on a
 * pseudo-random series of n elements (n = 0: 2^28).  Allocates and frees
 * its buffers (about 3 n elements plus the batches), leaves the stream's
 * 2-D scratch images in place, and synchronises `stream`; results of every
 * call stay bit-identical whatever it picks.  Not during graph capture
 * (EBUSY).  Calls made concurrently on other threads may see the table
 * change midway (each launch reads it once).
 * Errors: EINVAL for an unknown dtype or 0 < n < 2^20; ENOMEM.
 */
int maxmin_autotune(int dtype, int64_t n, void* stream);

/*
 * maxmin_tuning -- the current table for `dtype`, MAXMIN_TUNING_LEN entries:
 *   [0] tile run, w <= 2048 (sub-tiles)   [1] tile run, 2048 < w <= 8192
 *   [2] 2-D row-pass run (sub-tiles)      [3] ticket ranges, one-chunk windows
 *   [4] ticket ranges, look-back kernel   [5] strategy for w > 8192
 *                                             (MAXMIN_STRATEGY_CHUNK or _RUN)
 *   [6] batched tile (sub-tiles)
 *   [7 + 3 wc + nc] batched strategy of size class (wc, nc): 0 tile kernel,
 *       1 chunk kernel; wc = 0, 1, 2 for w <= 2048, <= 4096, <= 8192;
 *       nc = 0, 1, 2 for n < 2^16, < 2^20, longer (longer windows always
 *       take the chunk kernel)
 *   [16] 1 if measured by maxmin_autotune, else 0 (the built-in defaults).
 * Host only.
 */
#define MAXMIN_TUNING_LEN 17
int maxmin_tuning(int dtype, int64_t* out);

/* Grey-scale morphology operators of maxmin_morph_2d. */
typedef enum {
  MAXMIN_ERODE = 0,  /* min over the rectangle (the min half of maxmin_filter_2d) */
  MAXMIN_DILATE = 1, /* max over the rectangle */
  MAXMIN_OPEN = 2,   /* dilation of the erosion */
  MAXMIN_CLOSE = 3   /* erosion of the dilation */
} maxmin_morph_t;

/*
 * maxmin_morph_2d -- erosion, dilation, opening or closing of an image with
 * a w_rows x w_cols rectangle (Section 1: the filter's image-processing use,
 * applied to rows then columns), valid windows only.
 *   erode / dilate : output (rows-w_rows+1) x (cols-w_cols+1);
 *   open / close   : output (rows-2*w_rows+2) x (cols-2*w_cols+2) (two
 *                    filters; the intermediate image lives in library
 *                    scratch, grown outside graph capture).
 *   d_out : leading dimension ld_out (elements), caller-owned.
 * Errors: EINVAL for an unknown op, a window < 1, negative sizes,
 * ld_in < cols, ld_out < output width, or a null / misaligned pointer with
 * work to do; ENOMEM if scratch cannot be allocated.
 */
int maxmin_morph_2d(int dtype, const void* d_in, int64_t rows, int64_t cols, int64_t ld_in,
                    int64_t w_rows, int64_t w_cols, int op, void* d_out, int64_t ld_out,
                    void* stream);

/*
 * Serving engine -- many callers submit filter requests and stream chunks
 * (host buffers); the engine admits them against an HBM budget, batches the
 * requests that have arrived into single launches (one per dtype and
 * strategy) on one of `n_lanes` HIP streams, overlaps batches on the device,
 * and reports each request's latency (submit to completion).  Stream carries
 * (the last w-1 samples, Section 1's zero-latency streaming) stay resident on
 * the device inside the budget.
 *
 * Buffers: h_in (n or m elements) and h_max/h_min (max(0, n-w+1) elements
 * for a filter, m for a push) are HOST pointers owned by the caller and must
 * stay valid until the request is returned by maxmin_engine_poll.  Use
 * pinned memory (hipHostMalloc, torch pin_memory): a batch moves the pinned
 * (mapped) buffers under 1 MiB of all its requests with one gather kernel
 * before its filter launches and one scatter kernel after them (a small
 * hipMemcpyAsync costs ~10 us of copy-engine time); larger buffers take one
 * hipMemcpyAsync each on the copy engines, and pageable buffers one
 * synchronous hipMemcpyAsync each.  Requests with no complete
 * window finish at once.  A request larger than the whole budget finishes
 * with ENOMEM.
 * Back-pressure: at most 4096 requests (environment
 * MAXMIN_ENGINE_MAX_PENDING) wait for admission; a submit beyond that
 * returns MAXMIN_EBUSY at once and nothing is queued (the replay call skips
 * such a request and gives it id -1).  MAXMIN_ENGINE_COPIES=memcpy makes
 * every buffer take hipMemcpyAsync, MAXMIN_ENGINE_COPY_MAX sets the
 * kernel-copy size limit in bytes (experiments, tests).
 *
 * maxmin_engine_create: budget >= 1 MiB (allocated up front), 1..16 lanes,
 *   max_batch >= 1 requests per lane batch.  Errors: EINVAL, ENOMEM, EDEVICE.
 * maxmin_engine_open_stream / close_stream: a stream of `dtype` with window w
 *   (close waits for its queued pushes).
 * maxmin_engine_submit_filter / submit_push: enqueue (thread-safe); *req_id
 *   receives the request id.  Pushes of one stream complete in order.
 * maxmin_engine_poll: up to `cap` finished requests since the last poll:
 *   ids, n_out (windows written), latency in seconds, status; *got = count.
 *   Status EDEVICE: the request's batch failed.  If its HIP calls failed, a
 *   push leaves its stream as it was before the push (the chunk may be
 *   pushed again).  If the batch's chunk-strategy kernels report a look-back
 *   wait that gave up (see maxmin_check_stream), every request of the batch
 *   fails and each stream pushed in it is broken: its later pushes finish
 *   with EDEVICE (close it and open a new one).
 *   Tests can force either case: environment MAXMIN_ENGINE_INJECT="launch:K"
 *   or "err:K" (read at maxmin_engine_create) makes the engine's K-th batch
 *   fail before enqueuing anything, or report the look-back error word set.
 * maxmin_engine_drain: wait until every submitted request has finished.
 * maxmin_engine_stats: MAXMIN_ENGINE_STATS_LEN entries = {submitted,
 *   finished, batches, rejected (larger than the budget), samples
 *   processed, budget bytes in use, peak bytes in use, pending, refused by
 *   back-pressure}.
 * maxmin_engine_replay: open-loop load generator: submit request i at
 *   at_s[i] seconds after the call (kind 0 filter with dtype/n/w, kind 1
 *   push of n samples on stream sid[i]); req_ids and the submission lag
 *   (seconds late) per request are optional outputs.
 * maxmin_engine_destroy: drain, stop the engine threads, free everything.
 */
typedef struct maxmin_engine maxmin_engine_t;
int maxmin_engine_create(int64_t hbm_budget_bytes, int n_lanes, int64_t max_batch, maxmin_engine_t** out);
int maxmin_engine_open_stream(maxmin_engine_t* eng, int dtype, int64_t w, int64_t* stream_id);
int maxmin_engine_close_stream(maxmin_engine_t* eng, int64_t stream_id);
int maxmin_engine_submit_filter(maxmin_engine_t* eng, int dtype, const void* h_in, int64_t n, int64_t w,
                                void* h_max, void* h_min, int64_t* req_id);
int maxmin_engine_submit_push(maxmin_engine_t* eng, int64_t stream_id, const void* h_chunk, int64_t m,
                              void* h_max, void* h_min, int64_t* req_id);
int maxmin_engine_poll(maxmin_engine_t* eng, int64_t* ids, int64_t* n_out, double* latency_s, int* status,
                       int64_t cap, int64_t* got);
int maxmin_engine_drain(maxmin_engine_t* eng);
#define MAXMIN_ENGINE_STATS_LEN 9
int maxmin_engine_stats(maxmin_engine_t* eng, int64_t* out);
int maxmin_engine_replay(maxmin_engine_t* eng, int64_t count, const double* at_s, const int* kind,
                         const int* dtype, const int64_t* n, const int64_t* w, const int64_t* sid,
                         const void* const* h_in, void* const* h_max, void* const* h_min,
                         int64_t* req_ids, double* lag_s);
int maxmin_engine_destroy(maxmin_engine_t* eng);

/* Force a strategy for subsequent 1-D calls from this process (AUTO restores
 * the planner).  Used by tests to check that every strategy gives the same
 * bits.  Errors: EINVAL on an unknown value. */
int maxmin_set_strategy(int strategy);

/* Strategy the planner would use for (dtype, n, w): a maxmin_strategy_t. */
int maxmin_plan(int dtype, int64_t n, int64_t w);

/* Path maxmin_filter_2d takes for (dtype, w_rows, w_cols) with `outputs`
 * (2: max and min; 1: one of them null): MAXMIN_2D_FUSED (one pass, no
 * intermediate images: w_rows < 16, or w_rows < 24 for 16-bit data with
 * both outputs, and w_cols <= 64 V + 1 with V = 4 for w_rows < 8, 2 for
 * w_rows < 16, else 1) or MAXMIN_2D_ROWS_COLS (rows, then columns through
 * two library-owned intermediate images).  EINVAL for an unknown dtype, a
 * window < 1 or outputs not 1 or 2.  Host only. */
enum { MAXMIN_2D_FUSED = 1, MAXMIN_2D_ROWS_COLS = 2 };
int maxmin_plan_2d(int dtype, int64_t w_rows, int64_t w_cols, int outputs);

/* Synchronise `stream` (void* hipStream_t) and check the library's device
 * status words for it: MAXMIN_EDEVICE if a chunk-strategy look-back wait on
 * that stream ever gave up (its results are then invalid; not expected in
 * normal operation), else MAXMIN_OK. */
int maxmin_check_stream(void* stream);

/* Thread-local description of the last error ("" if none). */
const char* maxmin_last_error(void);

/* Library version string. */
const char* maxmin_version(void);

#ifdef __cplusplus
}
#endif

#endif /* MAXMIN_H */
