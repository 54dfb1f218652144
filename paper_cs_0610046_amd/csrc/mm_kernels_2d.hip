// gfx950 column passes of the 2-D filter (Section 1: the 1-D filter applied
// to rows, then to columns).  The row pass is the 1-D kernels' "rows" job
// into two row-filtered images; these kernels filter the columns of the max
// image (maxima) and of the min image (minima).  Both use van Herk /
// Gil-Werman blocks of exactly w_r rows, where the window that starts at
// row i of a block is
//     max(SUF[i], PRE[i + w_r - 1]) over that block and the next.
//
// k_cols: one wavefront per 64 columns and block of output rows, the
// block's suffixes in LDS (or global scratch past 64 KiB), then the next
// block's prefix top-down; every block of rows is read twice (as a block
// and as the next one).  It serves float64 and windows over 64 rows.
//
// k_cols_ring: one wavefront per strip of columns, band of output rows and
// image, streaming down the band with each column's current block in an LDS
// ring: every row is read once (plus w_r - 1 rows per band).
#include <algorithm>
#include <cstdlib>
#include <type_traits>

#include "mm_f2d.hpp"
#include "mm_launch.hpp"

namespace mm {

constexpr int kColBatch = 8;

// The block's suffix values live in LDS when 2 x 64 x w_rows elements fit in
// 64 KiB (GLOBAL_S = false), else in a global scratch slice owned by this
// wavefront.  The two are separate instantiations so that each pointer has
// one address space: an LDS pointer that may also point to global memory
// becomes a flat pointer, and flat LDS stores whose base register falls
// below the LDS aperture (as unrolled negative offsets produce) fault.
template <class T, bool GLOBAL_S>
__global__ __launch_bounds__(64) void k_cols(const T* __restrict__ M, const T* __restrict__ N, int64_t ld_t,
                                             int64_t rows, int64_t oc, int64_t w, T* __restrict__ omax,
                                             T* __restrict__ omin, int64_t ld_out, T* __restrict__ gscratch) {
  extern __shared__ unsigned char smem_raw[];
  T* Sx;
  if constexpr (GLOBAL_S)
    Sx = gscratch + ((int64_t)blockIdx.y * gridDim.x + blockIdx.x) * (2 * 64 * w);
  else
    Sx = reinterpret_cast<T*>(smem_raw);  // [w][64]
  T* Sn = Sx + 64 * w;
  const int lane = threadIdx.x;
  // M (and omax) or N (and omin) is null for a min-only / max-only filter
  const bool hx = M != nullptr, hn = N != nullptr;
  const int64_t c = (int64_t)blockIdx.x * 64 + lane;
  const bool act = c < oc;
  const int64_t cc = act ? c : 0;
  const int64_t orows = rows - w + 1;
  const int64_t r0 = (int64_t)blockIdx.y * w;  // first output row of the block
  if (r0 >= orows) return;
  const int64_t nb = min(w, orows - r0);  // outputs of this block

  // own block rows [r0, r0+w), bottom-up: suffix max/min
  T sx = Lim<T>::lo(), sn = Lim<T>::hi();
  for (int64_t i0 = w - 1; i0 >= 0; i0 -= kColBatch) {
    T vx[kColBatch], vn[kColBatch];
#pragma unroll
    for (int u = 0; u < kColBatch; ++u) {
      const int64_t i = i0 - u;
      vx[u] = Lim<T>::lo();
      vn[u] = Lim<T>::hi();
      if (i >= 0) {
        if (hx) vx[u] = M[(r0 + i) * ld_t + cc];
        if (hn) vn[u] = N[(r0 + i) * ld_t + cc];
      }
    }
#pragma unroll
    for (int u = 0; u < kColBatch; ++u) {
      const int64_t i = i0 - u;
      if (i >= 0) {
        sx = vmax(sx, vx[u]);
        sn = vmin(sn, vn[u]);
        Sx[i * 64 + lane] = sx;
        Sn[i * 64 + lane] = sn;
      }
    }
  }
  if (act) {
    if (hx) omax[r0 * ld_out + c] = sx;  // window r0 is exactly the block
    if (hn) omin[r0 * ld_out + c] = sn;
  }
  // next block, top-down: prefix max/min over rows r0+w .. r0+w-1+i
  T px = Lim<T>::lo(), pn = Lim<T>::hi();
  for (int64_t i0 = 1; i0 < nb; i0 += kColBatch) {
    T vx[kColBatch], vn[kColBatch];
#pragma unroll
    for (int u = 0; u < kColBatch; ++u) {
      const int64_t i = i0 + u;
      vx[u] = Lim<T>::lo();
      vn[u] = Lim<T>::hi();
      if (i < nb) {
        if (hx) vx[u] = M[(r0 + w - 1 + i) * ld_t + cc];
        if (hn) vn[u] = N[(r0 + w - 1 + i) * ld_t + cc];
      }
    }
#pragma unroll
    for (int u = 0; u < kColBatch; ++u) {
      const int64_t i = i0 + u;
      if (i < nb) {
        px = vmax(px, vx[u]);
        pn = vmin(pn, vn[u]);
        if (act) {
          if (hx) omax[(r0 + i) * ld_out + c] = vmax(Sx[i * 64 + lane], px);
          if (hn) omin[(r0 + i) * ld_out + c] = vmin(Sn[i * 64 + lane], pn);
        }
      }
    }
  }
}

template hipError_t f2d_launch<false, 3>(int, const void*, const void*, int64_t, int64_t, int64_t, int64_t, int64_t,
                                         void*, void*, int64_t, int64_t, hipStream_t);
template hipError_t f2d_launch<true, 3>(int, const void*, const void*, int64_t, int64_t, int64_t, int64_t, int64_t,
                                        void*, void*, int64_t, int64_t, hipStream_t);

bool f2d_eligible(int dtype, int64_t w_rows, int64_t w_cols) {
  if (dtype < 0 || dtype > 3 || w_rows < 1 || w_rows > 64 || w_cols < 1) return false;
  int B = 1;
  while (2 * B <= w_rows) B *= 2;
  return w_cols <= 64 * f2d_V(B, f2d_size(dtype)) + 1;
}

hipError_t launch_f2d(int dtype, const void* d_in, int64_t ld_in, int64_t rows, int64_t cols, int64_t w_rows,
                      int64_t w_cols, void* d_max, void* d_min, int64_t ld_out, int64_t band_rows, hipStream_t st) {
  if (!f2d_eligible(dtype, w_rows, w_cols)) return hipErrorNotSupported;
  if (!d_max && !d_min) return hipErrorInvalidValue;
  auto* f = !d_min ? &f2d_launch<false, 1> : (!d_max ? &f2d_launch<false, 2> : &f2d_launch<false, 3>);
  return f(dtype, d_in, d_in, ld_in, rows, cols, w_rows, w_cols, d_max, d_min, ld_out, band_rows, st);
}

hipError_t launch_f2d_cols(int dtype, const void* tmax, const void* tmin, int64_t ld_t, int64_t rows, int64_t oc,
                           int64_t w_rows, void* d_max, void* d_min, int64_t ld_out, int64_t band_rows,
                           hipStream_t st) {
  if (dtype < 0 || dtype > 3 || w_rows < 1 || w_rows > 64) return hipErrorNotSupported;
  if (!tmax && !tmin) return hipErrorInvalidValue;
  if ((tmax == nullptr) != (d_max == nullptr) || (tmin == nullptr) != (d_min == nullptr)) return hipErrorInvalidValue;
  // a missing image (one output only) is never read; its pointer repeats
  // the other one's so the alignment test covers a real address
  const void* a = tmax ? tmax : tmin;
  const void* b = tmin ? tmin : tmax;
  auto* f = !d_min ? &f2d_launch<true, 1> : (!d_max ? &f2d_launch<true, 2> : &f2d_launch<true, 3>);
  return f(dtype, a, b, ld_t, rows, oc, w_rows, 1, d_max, d_min, ld_out, band_rows, st);
}

// Column pass streaming down a band of output rows, each column's block
// kept in an LDS ring of w_rows slots (w_rows <= 64; 4-byte data one column
// per lane, 16-bit data two adjacent columns per lane packed in one 32-bit
// slot).  A wavefront filters one image (the max image for maxima or the
// min image for minima): the two are independent, and one ring per
// wavefront (w_rows x 256 bytes) leaves room for ten wavefronts per CU.
// Blocks of exactly w_rows rows: the band's first block is loaded into the
// ring and turned into its suffixes; every later row i of a block is folded
// into the running prefix, emits the window that starts one row below the
// block above's row i,
//     out = max(SUF[i + 1], PRE),
// and takes slot i, the slot that was just read for the last time; at the
// block's end the ring turns into the new block's suffixes.  Each input row
// is read once (plus w_rows - 1 rows at the top of every band), so the
// images are not read twice as by the one-block-per-wavefront form.
// (A register ring indexed by the uniform row number made the compiler copy
// half the ring per access.)
template <class L> __device__ __forceinline__ uint32_t rg_bits(L v) {
  if constexpr (std::is_same_v<L, P16>) return v.v;
  else return __builtin_bit_cast(uint32_t, v);
}
template <class L> __device__ __forceinline__ L rg_val(uint32_t b) {
  if constexpr (std::is_same_v<L, P16>) return P16{b};
  else return __builtin_bit_cast(L, b);
}
template <class L, bool MAXF> __device__ __forceinline__ L rg_sel(L a, L b) {
  if constexpr (std::is_same_v<L, P16>) return MAXF ? hmax(a, b) : hmin(a, b);
  else return MAXF ? vmax(a, b) : vmin(a, b);
}
// A lane's V words of one row (V lane values: 4-byte elements, or pairs of
// 16-bit elements), moved with one V-word access.
template <int V> struct RgW {
  uint32_t u[V];
};
template <int V> __device__ __forceinline__ RgW<V> rg_gload(const uint32_t* p) {
  RgW<V> r;
  if constexpr (V == 1) {
    r.u[0] = gload(p);
  } else if constexpr (V == 2) {
    const f2_u32x2 t = gload((const f2_u32x2*)p);
    r.u[0] = t[0];
    r.u[1] = t[1];
  } else {
    static_assert(V == 4, "1, 2 or 4 words per lane");
    const f2_u32x4 t = gload((const f2_u32x4*)p);
#pragma unroll
    for (int j = 0; j < 4; ++j) r.u[j] = t[j];
  }
  return r;
}
template <int V> __device__ __forceinline__ RgW<V> rg_lds_get(const uint32_t* p) {
  RgW<V> r;
  if constexpr (V == 1) {
    r.u[0] = p[0];
  } else if constexpr (V == 2) {
    const f2_u32x2 t = *(const f2_u32x2*)p;
    r.u[0] = t[0];
    r.u[1] = t[1];
  } else {
    const f2_u32x4 t = *(const f2_u32x4*)p;
#pragma unroll
    for (int j = 0; j < 4; ++j) r.u[j] = t[j];
  }
  return r;
}
template <int V> __device__ __forceinline__ void rg_lds_put(uint32_t* p, const RgW<V>& r) {
  if constexpr (V == 1) {
    p[0] = r.u[0];
  } else if constexpr (V == 2) {
    f2_u32x2 t;
    t[0] = r.u[0];
    t[1] = r.u[1];
    *(f2_u32x2*)p = t;
  } else {
    f2_u32x4 t;
#pragma unroll
    for (int j = 0; j < 4; ++j) t[j] = r.u[j];
    *(f2_u32x4*)p = t;
  }
}
template <class L, bool MAXF, int V> __device__ __forceinline__ RgW<V> rg_selw(const RgW<V>& a, const RgW<V>& b) {
  RgW<V> r;
#pragma unroll
  for (int j = 0; j < V; ++j) r.u[j] = rg_bits(rg_sel<L, MAXF>(rg_val<L>(a.u[j]), rg_val<L>(b.u[j])));
  return r;
}
// The ring's raw block (slots 0..w-1; slot k of this lane at ring[64 V k])
// -> its suffixes (slot k: the selection over rows k..w-1); eight slots
// read per batch so that their latencies overlap.
template <class L, bool MAXF, int V> __device__ __forceinline__ void rg_suffixes(uint32_t* ring, int w) {
  RgW<V> acc;
#pragma unroll
  for (int j = 0; j < V; ++j) acc.u[j] = rg_bits(MAXF ? Lim<L>::lo() : Lim<L>::hi());
  for (int k0 = w - 1; k0 >= 0; k0 -= 8) {
    RgW<V> t[8];
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (k0 - u >= 0) t[u] = rg_lds_get<V>(ring + 64 * V * (k0 - u));
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      if (k0 - u >= 0) {
        acc = rg_selw<L, MAXF, V>(acc, t[u]);
        rg_lds_put<V>(ring + 64 * V * (k0 - u), acc);
      }
    }
  }
}
// One output row of the lane: its V words = V * H elements from column c
// (one V-word store where all of them exist and the address allows it).
template <class L, int V>
__device__ __forceinline__ void rg_store(typename F2Store<L>::S* p, int64_t c, int64_t oc, const RgW<V>& y) {
  using S = typename F2Store<L>::S;
  constexpr int H = F2Store<L>::halves;
  if (c + V * H <= oc && ((uintptr_t)p & (4 * V - 1)) == 0) {
    if constexpr (V == 1) {
      gstore((uint32_t*)p, y.u[0]);
    } else if constexpr (V == 2) {
      f2_u32x2 t;
      t[0] = y.u[0];
      t[1] = y.u[1];
      gstore((f2_u32x2*)p, t);
    } else {
      f2_u32x4 t;
#pragma unroll
      for (int j = 0; j < 4; ++j) t[j] = y.u[j];
      gstore((f2_u32x4*)p, t);
    }
    return;
  }
#pragma unroll
  for (int j = 0; j < V * H; ++j) {
    if (c + j < oc) {
      const uint32_t word = y.u[j / H];
      if constexpr (H == 2) gstore(p + j, (S)(j % 2 ? word >> 16 : word & 0xFFFFu));
      else gstore(p + j, __builtin_bit_cast(S, word));
    }
  }
}

// ldl: row stride of the row-filtered image in 32-bit words; band: output
// rows per wavefront, a multiple of w.  Each lane owns V words of a row.
template <class L, bool MAXF, int D, int V>
__device__ __forceinline__ void cols_ring_body(const uint32_t* __restrict__ X, int64_t ldl, int64_t rows, int64_t oc,
                                               int w, int64_t band, typename F2Store<L>::S* __restrict__ out,
                                               int64_t ld_out, uint32_t* ring) {
  constexpr int H = F2Store<L>::halves;  // image columns per word
  const int lane = threadIdx.x;
  const int64_t cw = ((int64_t)blockIdx.x * 64 + lane) * V;  // first word of the lane
  const int64_t c = cw * H;                                  // first image column of the lane
  const int64_t ccw = c < oc ? cw : 0;                       // lanes past the edge load word 0
  const int64_t orows = rows - w + 1;
  const int64_t o0 = (int64_t)blockIdx.y * band;
  if (o0 >= orows) return;
  const int64_t nb = min(band, orows - o0);  // outputs of this band
  const int64_t rlast = o0 + nb + w - 2;     // last input row it needs
  const uint32_t* src = X + ccw;
  auto* q = out + c;
  ring += lane * V;

  // Rows go in groups of at most D that never cross a block's end (group
  // at position g0 of its block: min(D, w - g0) rows).  The next group's
  // rows load while this one runs, and this group's ring slots are read
  // together at its start (each slot is read before the row that takes it).
  RgW<V> buf[D];
#pragma unroll
  for (int d = 0; d < D; ++d) buf[d] = rg_gload<V>(src + min(o0 + d, rlast) * ldl);
  RgW<V> run;
  int64_t gs = o0;    // first row of the group
  int g0 = 0;         // its position in its block
  bool first = true;  // still loading the band's first block
  while (gs <= rlast) {
    const int len = min(D, w - g0);
    const int64_t ngs = gs + len;
    RgW<V> v[D];
#pragma unroll
    for (int d = 0; d < D; ++d) {
      v[d] = buf[d];
      buf[d] = rg_gload<V>(src + min(ngs + d, rlast) * ldl);
    }
    if (first) {
#pragma unroll
      for (int d = 0; d < D; ++d)
        if (d < len) rg_lds_put<V>(ring + 64 * V * (g0 + d), v[d]);
    } else {
      RgW<V> sf[D];
#pragma unroll
      for (int d = 0; d < D; ++d)
        if (d < len && g0 + d + 1 < w) sf[d] = rg_lds_get<V>(ring + 64 * V * (g0 + d + 1));
#pragma unroll
      for (int d = 0; d < D; ++d) {
        const int64_t r = gs + d;
        if (d >= len || r > rlast) break;
        const int i = g0 + d;
        run = i == 0 ? v[d] : rg_selw<L, MAXF, V>(run, v[d]);
        const RgW<V> y = i < w - 1 ? rg_selw<L, MAXF, V>(sf[d], run) : run;
        rg_store<L, V>(q + (r - w + 1) * ld_out, c, oc, y);  // the window this row completes
        rg_lds_put<V>(ring + 64 * V * i, v[d]);
      }
    }
    if (g0 + len == w) {  // the block is complete
      if (first || ngs - 1 < rlast) rg_suffixes<L, MAXF, V>(ring, w);
      // the band's first window is exactly its first block
      if (first) rg_store<L, V>(q + o0 * ld_out, c, oc, rg_lds_get<V>(ring));
      first = false;
      g0 = 0;
    } else {
      g0 += len;
    }
    gs = ngs;
  }
}

// blockIdx.z == 0: max-filter M into omax (when it is not null), else
// min-filter N into omin.  Dynamic LDS: w x 64 x V words.  D: rows of loads
// in flight per wavefront.
template <class L, int D, int V>
__global__ __launch_bounds__(64) void k_cols_ring(const uint32_t* __restrict__ M, const uint32_t* __restrict__ N,
                                                  int64_t ldl, int64_t rows, int64_t oc, int w, int64_t band,
                                                  typename F2Store<L>::S* __restrict__ omax,
                                                  typename F2Store<L>::S* __restrict__ omin, int64_t ld_out) {
  extern __shared__ uint32_t rg_ring[];
  if (blockIdx.z == 0 && omax)
    cols_ring_body<L, true, D, V>(M, ldl, rows, oc, w, band, omax, ld_out, rg_ring);
  else
    cols_ring_body<L, false, D, V>(N, ldl, rows, oc, w, band, omin, ld_out, rg_ring);
}

static int cols_cus() {
  static int cus = 0;
  if (!cus) {
    int dev = 0;
    (void)hipGetDevice(&dev);
    hipDeviceProp_t p;
    if (hipGetDeviceProperties(&p, dev) == hipSuccess) cus = p.multiProcessorCount;
    if (cus <= 0) cus = 256;
  }
  return cus;
}

hipError_t launch_cols_ring(int dtype, const void* tmax, const void* tmin, int64_t ld_t, int64_t rows, int64_t oc,
                            int64_t wr, void* d_max, void* d_min, int64_t ld_out, int64_t band_rows,
                            hipStream_t st) {
  if (dtype == 1 || dtype < 0 || dtype > 3 || wr < 1 || wr > 64) return hipErrorNotSupported;
  if (!tmax && !tmin) return hipErrorInvalidValue;
  if ((tmax == nullptr) != (d_max == nullptr) || (tmin == nullptr) != (d_min == nullptr)) return hipErrorInvalidValue;
  const int64_t orows = rows - wr + 1;
  if (orows <= 0 || oc <= 0) return hipSuccess;
  const int H = dtype == 3 ? 2 : 1;  // elements per 32-bit word
  // Words per lane V, rows in flight D and blocks per band: on MI355X
  // (8192^2, rows then columns, whole call) float32 w = 16 / 31 took 0.42 /
  // 0.45 ms with V = 2 (0.48 / 0.49 with the fused kernel's column filter),
  // w = 63 0.51 with V = 1 (the same); uint16 w = 16 / 31 0.29 / 0.30 with
  // V = 2 and w = 63 0.32 with V = 1 (0.30 / 0.32 / 0.42 before).  Bands of
  // a fixed number of blocks beat bands sized to hold the grid at once
  // (f32 w = 63: 0.51 against 0.65 ms); they shrink only where the grid
  // would fall under four wavefronts per CU.  MAXMIN_COLS_V / _D set V and
  // D (experiments, tests).
  int V = H == 2 ? (wr > 32 ? 1 : 2) : (wr > 48 ? 1 : 2);
  int64_t nb_pref = H == 2 ? 8 : (V == 1 ? 16 : 4);
  const char* ev = getenv("MAXMIN_COLS_V");
  if (ev) V = atoi(ev) >= 4 ? 4 : atoi(ev) >= 2 ? 2 : 1;
  // lanes load V words of a row at once: rows start on 4V-byte boundaries
  // and hold whole lane groups (ld_t a multiple of the lane's elements)
  const int64_t per_lane = (int64_t)V * H;
  if ((ld_t % per_lane) || ((uintptr_t)tmax % (4 * V)) || ((uintptr_t)tmin % (4 * V))) return hipErrorNotSupported;
  const int64_t ldl = ld_t / H;
  const int64_t lanes = (oc + per_lane - 1) / per_lane;
  const int64_t strips = (lanes + 63) / 64;
  const int64_t blocks = (orows + wr - 1) / wr;
  const size_t lds = (size_t)wr * 256 * V;
  const int64_t images = (d_max && d_min) ? 2 : 1;
  int64_t nblk;
  if (band_rows > 0) {
    nblk = std::max<int64_t>(1, band_rows / wr);
  } else {
    const int64_t min_waves = (int64_t)cols_cus() * 4;
    const int64_t bands_fill = (min_waves + strips * images - 1) / (strips * images);
    nblk = std::max<int64_t>(1, std::min<int64_t>(nb_pref, (blocks + bands_fill - 1) / bands_fill));
  }
  const int64_t band = nblk * wr;
  const int64_t nbands = (orows + band - 1) / band;
  if (strips > INT32_MAX || nbands > 65535) return hipErrorNotSupported;
  // one wavefront per strip, band and image
  const dim3 grid((unsigned)strips, (unsigned)nbands, (unsigned)images);
  const char* ed = getenv("MAXMIN_COLS_D");
  const int dd = ed ? atoi(ed) : 16;
  auto go = [&](auto* lp, auto* sp) {
    using L = std::remove_pointer_t<decltype(lp)>;
    using S = std::remove_pointer_t<decltype(sp)>;
    auto* f = &k_cols_ring<L, 8, 1>;
    if (V == 1) f = dd >= 16 ? &k_cols_ring<L, 16, 1> : &k_cols_ring<L, 8, 1>;
    else if (V == 2) f = dd >= 16 ? &k_cols_ring<L, 16, 2> : &k_cols_ring<L, 8, 2>;
    else f = &k_cols_ring<L, 8, 4>;
    hipLaunchKernelGGL(f, grid, dim3(64), lds, st, (const uint32_t*)tmax, (const uint32_t*)tmin, ldl, rows, oc,
                       (int)wr, band, (S*)d_max, (S*)d_min, ld_out);
    return hipGetLastError();
  };
  switch (dtype) {
    case 0: return go((float*)nullptr, (float*)nullptr);
    case 2: return go((int32_t*)nullptr, (int32_t*)nullptr);
    case 3: return go((P16*)nullptr, (uint16_t*)nullptr);
    default: return hipErrorNotSupported;
  }
}

int64_t cols_max_window(int dtype) {
  const int64_t s = dtype == 1 ? 8 : (dtype == 3 ? 2 : 4);
  return (64 * 1024) / (2 * 64 * s);  // LDS: 2 images x 64 columns x w rows <= 64 KiB
}

int64_t cols_scratch_elems(int64_t rows, int64_t oc, int64_t wr) {
  const int64_t orows = rows - wr + 1;
  if (orows <= 0 || oc <= 0) return 0;
  return ((oc + 63) / 64) * ((orows + wr - 1) / wr) * 2 * 64 * wr;
}

hipError_t launch_cols(int dtype, const void* tmax, const void* tmin, int64_t ld_t, int64_t rows, int64_t oc,
                       int64_t wr, void* d_max, void* d_min, int64_t ld_out, void* gscratch, hipStream_t st) {
  const int64_t orows = rows - wr + 1;
  if (orows <= 0 || oc <= 0) return hipSuccess;
  const dim3 grid((unsigned)((oc + 63) / 64), (unsigned)((orows + wr - 1) / wr));
  auto go = [&](auto* p) {
    using T = std::remove_pointer_t<decltype(p)>;
    if (gscratch)
      hipLaunchKernelGGL((k_cols<T, true>), grid, dim3(64), 0, st, (const T*)tmax, (const T*)tmin, ld_t, rows, oc,
                         wr, (T*)d_max, (T*)d_min, ld_out, (T*)gscratch);
    else
      hipLaunchKernelGGL((k_cols<T, false>), grid, dim3(64), (size_t)2 * 64 * wr * sizeof(T), st, (const T*)tmax,
                         (const T*)tmin, ld_t, rows, oc, wr, (T*)d_max, (T*)d_min, ld_out, (T*)nullptr);
    return hipGetLastError();
  };
  switch (dtype) {
    case 0: return go((float*)nullptr);
    case 1: return go((double*)nullptr);
    case 2: return go((int32_t*)nullptr);
    case 3: return go((uint16_t*)nullptr);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace mm
