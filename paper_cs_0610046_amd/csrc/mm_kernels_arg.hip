// gfx950 arg max/min filter for long windows (the locations the monotonic
// wedge keeps, Section 5): one step from the tile kernel's level of window
// q to the final window w.
//
// With F = ceil(w / 4096) and q = floor(w / F) <= 4096, the window [j, j+w)
// is the union of the F windows of length q starting at j, j+q, ...,
// j+(F-1)q (they cover [j, j+Fq)) and, when Fq < w, the one starting at
// j+w-q ((F+1)q >= w since w >= F^2 - 1).  Seen as a matrix with rows of q
// level entries, the first F are one column's F consecutive rows: a
// running window of F rows down every column, done like the 2-D column
// pass (van Herk/Gil-Werman with blocks of B rows, a per-lane LDS ring of
// 2B rows), so each level entry is read once instead of F times.
// Combining (value, location) pairs keeps the larger (smaller) value and,
// on ties, the smaller location: associative and commutative, so every
// grouping gives each window its leftmost max and min.
#include <algorithm>
#include <type_traits>

#include "mm_launch.hpp"

namespace mm {

template <class T> struct ArgColsArgs {
  const T* vx;  // level: max values, locations of the max, min values, locations of the min
  const int64_t* ix;
  const T* vn;
  const int64_t* in;
  int64_t nlv, q, w, nout;  // level entries, row width, final window, final outputs
  int F;
  T* ox;
  int64_t* jx;
  T* on;
  int64_t* jn;
  int64_t rows;  // output rows: ceil(nout / q)
  int strips, TR;
  int64_t ntiles;
};

template <class T, int B>
__global__ __launch_bounds__(64) void k_argcols(ArgColsArgs<T> a) {
  typedef Loc<T> E;
  constexpr int RB = 2 * B, D = 8;
  constexpr int lgB = B == 1 ? 0 : (B == 2 ? 1 : (B == 4 ? 2 : (B == 8 ? 3 : 4)));
  __shared__ E ringx[RB * 64], ringn[RB * 64];  // [slot][lane], private to each lane
  const int lane = threadIdx.x;
  const int64_t per = gridDim.x / 8;  // consecutive tiles on one XCD
  const int64_t tile = (int64_t)(blockIdx.x & 7) * per + (blockIdx.x >> 3);
  if (tile >= a.ntiles) return;
  const int64_t band = tile / a.strips, strip = tile - band * a.strips;
  const int64_t b = strip * 64 + lane;  // this lane's column
  if (b >= a.q) return;                 // lanes share nothing: an idle one just leaves
  const int64_t r0 = band * (int64_t)a.TR;
  const int nr = (int)min((int64_t)a.TR, a.rows - r0);
  const int F = a.F, NR = nr + F - 1;
  const int64_t base = r0 * a.q;  // locations are kept relative to it (int32)
  const bool extra = a.w > (int64_t)F * a.q;

  T qx[D], qn[D];
  int64_t lx[D], ln[D];
  auto load = [&](int t, int d) {
    const int64_t p = min((r0 + t) * a.q + b, a.nlv - 1);  // clamped rows feed no valid output
    qx[d] = gload(a.vx + p);
    lx[d] = gload(a.ix + p);
    qn[d] = gload(a.vn + p);
    ln[d] = gload(a.in + p);
  };
#pragma unroll
  for (int d = 0; d < D; ++d)
    if (d < NR) load(d, d);
  E Px = {Lim<T>::lo(), 0}, Pn = {Lim<T>::hi(), 0}, Ax = Px, An = Pn;
  for (int t0 = 0; t0 < NR; t0 += D) {
#pragma unroll
    for (int d = 0; d < D; ++d) {
      const int t = t0 + d;
      if (t < NR) {
        const E ex = {qx[d], (int)(lx[d] - base)}, en = {qn[d], (int)(ln[d] - base)};
        if (t + D < NR) load(t + D, d);
        const int slot = t & (RB - 1);
        if ((t & (B - 1)) == 0 && t > 0) {
          // the block before this row is complete: its suffixes, in place
          const int s0 = (t - B) & (RB - 1);
          E ux = ringx[(s0 + B - 1) * 64 + lane], un = ringn[(s0 + B - 1) * 64 + lane];
          for (int k = B - 2; k >= 0; --k) {
            const int ix = (s0 + k) * 64 + lane;
            ux = vmax(ux, ringx[ix]);
            un = vmin(un, ringn[ix]);
            ringx[ix] = ux;
            ringn[ix] = un;
          }
          Ax = ux;
          An = un;
        }
        const bool bstart = (t & (B - 1)) == 0;
        ringx[slot * 64 + lane] = ex;
        ringn[slot * 64 + lane] = en;
        Px = bstart ? ex : vmax(Px, ex);
        Pn = bstart ? en : vmin(Pn, en);
        if (t >= F - 1) {
          // the F rows [j, t] of this column are complete
          const int j = t - F + 1, bj = j >> lgB, bt = t >> lgB;
          E ox = Px, on = Pn;
          if (bt > bj) {
            ox = vmax(ox, ringx[(j & (RB - 1)) * 64 + lane]);
            on = vmin(on, ringn[(j & (RB - 1)) * 64 + lane]);
          }
          if (bt > bj + 1) {
            ox = vmax(ox, Ax);
            on = vmin(on, An);
          }
          const int64_t o = (r0 + j) * a.q + b;
          if (o < a.nout) {
            if (extra) {
              const int64_t p = o + a.w - a.q;
              ox = vmax(ox, E{gload(a.vx + p), (int)(gload(a.ix + p) - base)});
              on = vmin(on, E{gload(a.vn + p), (int)(gload(a.in + p) - base)});
            }
            gstore(a.ox + o, ox.v);
            gstore(a.jx + o, (int64_t)ox.i + base);
            gstore(a.on + o, on.v);
            gstore(a.jn + o, (int64_t)on.i + base);
          }
        }
      }
    }
  }
}

// ------------------------------------------------------------------
// Windows past the tile kernel's (w > 4096): blocks of exactly w inputs
// aligned at the series start, cut into K chunks of at most 2048 (the
// chunk decomposition of the plain filter), in two passes.  Pass 1
// (k_argagg): every chunk's max and min with their leftmost locations.
// Pass 2 (k_argcol): workgroup g walks column k = g mod K over a range of
// blocks; the windows ending in chunk (b, k) start in chunk (b-1, k), which
// it loaded one step before, so each window is the suffix of that chunk
// from its first element, the pass-1 aggregates of chunks (b-1, k+1..K-1)
// and (b, 0..k-1), and the prefix of chunk (b, k) to its last element.
// Locations travel as int32 offsets from the start of block b-1 (below
// 2w), and every combine prefers the smaller location on equal values, so
// each window gets its leftmost max and min whatever the grouping.  The
// input is read twice and each output written once.
constexpr int kArgThreads = 256;
constexpr int kArgV = 8;
constexpr int64_t kArgChunk = int64_t(kArgThreads) * kArgV;  // 2048
typedef unsigned int ag_u32x4 __attribute__((ext_vector_type(4)));

template <class T> __device__ __forceinline__ Loc<T> loc_lo() { return Loc<T>{Lim<T>::lo(), 0x7fffffff}; }
template <class T> __device__ __forceinline__ Loc<T> loc_hi() { return Loc<T>{Lim<T>::hi(), 0x7fffffff}; }

// V inputs of chunk slots r0 .. r0+V-1 at p (slots >= len read as 0, never used)
template <class T>
__device__ __forceinline__ void arg_load(const T* p, int r0, int len, T (&v)[kArgV]) {
  constexpr int EV = 16 / (int)sizeof(T);
  if (r0 + kArgV <= len && ((uintptr_t)(p + r0) & 15) == 0) {
#pragma unroll
    for (int k = 0; k < kArgV / EV; ++k) {
      const ag_u32x4 u = gload((const ag_u32x4*)(p + r0 + k * EV));
      __builtin_memcpy(&v[k * EV], &u, 16);
    }
  } else {
#pragma unroll
    for (int i = 0; i < kArgV; ++i) v[i] = r0 + i < len ? gload(p + r0 + i) : T(0);
  }
}

template <class T>
__device__ __forceinline__ void arg_chunk_geom(int64_t w, int64_t& K, int64_t& C) {
  K = (w + kArgChunk - 1) / kArgChunk;
  C = (w + K - 1) / K;
}

template <class T>
__global__ __launch_bounds__(kArgThreads) void k_argagg(const T* __restrict__ a, int64_t n, int64_t w,
                                                        T* __restrict__ avx, int* __restrict__ aix,
                                                        T* __restrict__ avn, int* __restrict__ ain) {
  __shared__ Loc<T> red[2][kArgThreads / 64];
  int64_t K, C;
  arg_chunk_geom<T>(w, K, C);
  const int64_t NB = (n + w - 1) / w, nch = NB * K;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, r0 = tid * kArgV;
  for (int64_t t = blockIdx.x; t < nch; t += gridDim.x) {
    const int64_t b = t / K, k = t - b * K;
    const int64_t p0 = b * w + k * C;
    const int len = p0 < n ? (int)min(min(C, w - k * C), n - p0) : 0;
    T v[kArgV];
    arg_load<T>(a + min(p0, n - 1), r0, len, v);
    Loc<T> mx = loc_lo<T>(), mn = loc_hi<T>();
#pragma unroll
    for (int i = 0; i < kArgV; ++i)
      if (r0 + i < len) {
        const Loc<T> e{v[i], (int)(k * C) + r0 + i};
        mx = vmax(mx, e);
        mn = vmin(mn, e);
      }
    for (int d = 32; d >= 1; d >>= 1) {
      mx = vmax(mx, Loc<T>{(T)__shfl_xor(mx.v, d, 64), __shfl_xor(mx.i, d, 64)});
      mn = vmin(mn, Loc<T>{(T)__shfl_xor(mn.v, d, 64), __shfl_xor(mn.i, d, 64)});
    }
    if (lane == 0) {
      red[0][wave] = mx;
      red[1][wave] = mn;
    }
    __syncthreads();
    if (tid == 0) {
      for (int q = 1; q < kArgThreads / 64; ++q) {
        mx = vmax(mx, red[0][q]);
        mn = vmin(mn, red[1][q]);
      }
      avx[t] = mx.v;
      aix[t] = mx.i;
      avn[t] = mn.v;
      ain[t] = mn.i;
    }
    __syncthreads();
  }
}

template <class T> struct ArgColLds {
  T xs[lds_len<T>(kArgChunk)];        // staged max values
  T hs[lds_len<T>(kArgChunk)];        // staged min values
  int lx[lds_len<int>(kArgChunk)];    // staged max locations (offsets from block b-1)
  int ln[lds_len<int>(kArgChunk)];    // staged min locations
  Loc<T> red[4][kArgThreads / 64];    // per-wave scan totals
  Loc<T> dep[4];                      // aggregates: PRE side max / min, SUF side max / min
  T edge[kArgThreads / 64];
};

template <class T>
__global__ __launch_bounds__(kArgThreads) void k_argcol(const T* __restrict__ a, int64_t n, int64_t w,
                                                        const T* __restrict__ avx, const int* __restrict__ aix,
                                                        const T* __restrict__ avn, const int* __restrict__ ain,
                                                        T* __restrict__ ox, int64_t* __restrict__ jx,
                                                        T* __restrict__ on, int64_t* __restrict__ jn) {
  constexpr int V = kArgV, NW = kArgThreads / 64;
  __shared__ ArgColLds<T> sm;
  int64_t K, C;
  arg_chunk_geom<T>(w, K, C);
  const int64_t NB = (n + w - 1) / w;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, r0 = tid * V;
  const int64_t k = blockIdx.x % K, R = gridDim.x / K, rr = blockIdx.x / K;
  const int64_t per = (NB + R - 1) / R;
  const int64_t b0 = rr * per, b1 = min(NB, b0 + per);
  const int lenfull = (int)min(C, w - k * C);
  if (b0 >= b1 || b0 * w + k * C >= n) return;
  T prev[V], cur[V];
#pragma unroll
  for (int i = 0; i < V; ++i) prev[i] = T(0);
  if (b0 >= 1) arg_load<T>(a + (b0 - 1) * w + k * C, r0, lenfull, prev);  // whole: it ends before block b0
  arg_load<T>(a + b0 * w + k * C, r0, (int)min((int64_t)lenfull, n - (b0 * w + k * C)), cur);
  for (int64_t b = b0; b < b1; ++b) {
    const int64_t p0 = b * w + k * C;
    if (p0 >= n) break;
    const int len = (int)min((int64_t)lenfull, n - p0);
    T nxt[V];
#pragma unroll
    for (int i = 0; i < V; ++i) nxt[i] = T(0);
    const int64_t p1 = p0 + w;
    if (b + 1 < b1 && p1 < n) arg_load<T>(a + p1, r0, (int)min((int64_t)lenfull, n - p1), nxt);
    const bool has_out = (p0 + len - 1) >= (w - 1);
    const int kc = (int)(k * C);
    // aggregates of the chunks between (pass 1), loaded ahead of the scans
    Loc<T> gx0 = loc_lo<T>(), gn0 = loc_hi<T>(), gx1 = loc_lo<T>(), gn1 = loc_hi<T>();
    if (has_out && tid < 64) {
      for (int64_t j = tid; j < K; j += 64) {
        if (j < k) {
          const int64_t q = b * K + j;
          gx0 = vmax(gx0, Loc<T>{avx[q], (int)w + aix[q]});
          gn0 = vmin(gn0, Loc<T>{avn[q], (int)w + ain[q]});
        } else if (j > k && b >= 1) {
          const int64_t q = (b - 1) * K + j;
          gx1 = vmax(gx1, Loc<T>{avx[q], aix[q]});
          gn1 = vmin(gn1, Loc<T>{avn[q], ain[q]});
        }
      }
    }
    // behind slot r: the previous chunk's slot r + 1, from this lane, the
    // next lane, or the next wavefront's lane 0
    if (lane == 0) sm.edge[wave] = prev[0];
    __syncthreads();
    T nb = __shfl_down(prev[0], 1, 64);
    if (lane == 63) nb = wave + 1 < NW ? sm.edge[wave + 1] : T(0);
    Loc<T> ax[V], an[V], bx[V], bn[V];
    const bool behind = b >= 1;
#pragma unroll
    for (int i = 0; i < V; ++i) {
      const int r = r0 + i;
      const Loc<T> e{cur[i], (int)w + kc + r};
      ax[i] = r < len ? e : loc_lo<T>();
      an[i] = r < len ? e : loc_hi<T>();
      const T h = i + 1 < V ? prev[i + 1 < V ? i + 1 : 0] : nb;
      const Loc<T> f{h, kc + r + 1};
      const bool vb = behind && r + 1 < lenfull;
      bx[i] = vb ? f : loc_lo<T>();
      bn[i] = vb ? f : loc_hi<T>();
    }
#pragma unroll
    for (int i = 1; i < V; ++i) {
      ax[i] = vmax(ax[i - 1], ax[i]);
      an[i] = vmin(an[i - 1], an[i]);
    }
#pragma unroll
    for (int i = V - 2; i >= 0; --i) {
      bx[i] = vmax(bx[i + 1], bx[i]);
      bn[i] = vmin(bn[i + 1], bn[i]);
    }
    // lane totals: inclusive prefix (own chunk) and suffix (previous chunk)
    // over the wavefront, then over the workgroup
    Loc<T> px = ax[V - 1], pn = an[V - 1], sx = bx[0], sn = bn[0];
    for (int d = 1; d < 64; d <<= 1) {
      const Loc<T> ux = shup(px, d, 64), un = shup(pn, d, 64);
      const Loc<T> vx = shdn(sx, d, 64), vn = shdn(sn, d, 64);
      if (lane >= d) {
        px = vmax(px, ux);
        pn = vmin(pn, un);
      }
      if (lane + d < 64) {
        sx = vmax(sx, vx);
        sn = vmin(sn, vn);
      }
    }
    if (lane == 63) {
      sm.red[0][wave] = px;
      sm.red[1][wave] = pn;
    }
    if (lane == 0) {
      sm.red[2][wave] = sx;
      sm.red[3][wave] = sn;
    }
    if (has_out && tid < 64) {
      for (int d = 32; d >= 1; d >>= 1) {
        gx0 = vmax(gx0, Loc<T>{(T)__shfl_xor(gx0.v, d, 64), __shfl_xor(gx0.i, d, 64)});
        gn0 = vmin(gn0, Loc<T>{(T)__shfl_xor(gn0.v, d, 64), __shfl_xor(gn0.i, d, 64)});
        gx1 = vmax(gx1, Loc<T>{(T)__shfl_xor(gx1.v, d, 64), __shfl_xor(gx1.i, d, 64)});
        gn1 = vmin(gn1, Loc<T>{(T)__shfl_xor(gn1.v, d, 64), __shfl_xor(gn1.i, d, 64)});
      }
      if (tid == 0) {
        sm.dep[0] = gx0;
        sm.dep[1] = gn0;
        sm.dep[2] = gx1;
        sm.dep[3] = gn1;
      }
    }
    __syncthreads();
    if (has_out) {
      // exclusive lane prefix / suffix: the lanes before (after) this one,
      // the wavefronts before (after) this one, and the aggregates
      Loc<T> cx = sm.dep[0], cn = sm.dep[1], ex = sm.dep[2], en = sm.dep[3];
      for (int q = 0; q < NW; ++q) {
        if (q < wave) {
          cx = vmax(cx, sm.red[0][q]);
          cn = vmin(cn, sm.red[1][q]);
        }
        if (q > wave) {
          ex = vmax(ex, sm.red[2][q]);
          en = vmin(en, sm.red[3][q]);
        }
      }
      const Loc<T> ux = shup(px, 1, 64), un = shup(pn, 1, 64);
      const Loc<T> vx = shdn(sx, 1, 64), vn = shdn(sn, 1, 64);
      if (lane > 0) {
        cx = vmax(cx, ux);
        cn = vmin(cn, un);
      }
      if (lane < 63) {
        ex = vmax(ex, vx);
        en = vmin(en, vn);
      }
#pragma unroll
      for (int i = 0; i < V; ++i) {
        const int r = r0 + i;
        if (r < len) {
          const Loc<T> mx = vmax(vmax(bx[i], ex), vmax(cx, ax[i]));
          const Loc<T> mn = vmin(vmin(bn[i], en), vmin(cn, an[i]));
          sm.xs[lds_idx<T>(r)] = mx.v;
          sm.hs[lds_idx<T>(r)] = mn.v;
          sm.lx[lds_idx<int>(r)] = mx.i;
          sm.ln[lds_idx<int>(r)] = mn.i;
        }
      }
    }
    __syncthreads();
    if (has_out) {
      const int rs = (int)max((int64_t)0, (w - 1) - p0);  // first slot whose window starts at >= 0
      const int64_t o = p0 - w + 1, base = (b - 1) * w;
      for (int r = rs + tid; r < len; r += kArgThreads) {
        ox[o + r] = sm.xs[lds_idx<T>(r)];
        on[o + r] = sm.hs[lds_idx<T>(r)];
        jx[o + r] = base + sm.lx[lds_idx<int>(r)];
        jn[o + r] = base + sm.ln[lds_idx<int>(r)];
      }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < V; ++i) {
      prev[i] = cur[i];
      cur[i] = nxt[i];
    }
  }
}

namespace {
int arg_cus() {
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
}  // namespace

size_t arg_chunk_scratch(int dtype, int64_t n, int64_t w) {
  const size_t s = dtype == 1 ? 8 : (dtype == 3 ? 2 : 4);
  const int64_t K = (w + kArgChunk - 1) / kArgChunk;
  const int64_t nch = ((n + w - 1) / w) * K;
  return (size_t)nch * 2 * (s + sizeof(int)) + 64;
}

hipError_t launch_arg_chunks(int dtype, const void* d_in, int64_t n, int64_t w, void* scratch, void* ox, int64_t* jx,
                             void* on, int64_t* jn, hipStream_t st) {
  if (n < w) return hipSuccess;
  if (w <= 1 || w > (int64_t(1) << 29)) return hipErrorInvalidValue;
  const int64_t K = (w + kArgChunk - 1) / kArgChunk;
  const int64_t nch = ((n + w - 1) / w) * K;
  auto go = [&](auto* p) -> hipError_t {
    using T = std::remove_pointer_t<decltype(p)>;
    T* avx = (T*)scratch;
    T* avn = avx + nch;
    int* aix = (int*)(((uintptr_t)(avn + nch) + 15) & ~(uintptr_t)15);
    int* ain = aix + nch;
    const int g1 = (int)std::min<int64_t>(nch, (int64_t)arg_cus() * 8);
    hipLaunchKernelGGL((k_argagg<T>), dim3(g1), dim3(kArgThreads), 0, st, (const T*)d_in, n, w, avx, aix, avn, ain);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_argcol<T>, kArgThreads, 0) != hipSuccess || nb < 1) nb = 1;
    const int64_t cap = (int64_t)nb * arg_cus();
    const int64_t g2 = std::max<int64_t>(1, cap / K) * K;
    if (g2 > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_argcol<T>), dim3((unsigned)g2), dim3(kArgThreads), 0, st, (const T*)d_in, n, w,
                       (const T*)avx, (const int*)aix, (const T*)avn, (const int*)ain, (T*)ox, jx, (T*)on, jn);
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

hipError_t launch_arg_cols(int dtype, const void* vx, const int64_t* ix, const void* vn, const int64_t* in,
                           int64_t nlv, int64_t q, int64_t w, int64_t nout, void* ox, int64_t* jx, void* on,
                           int64_t* jn, hipStream_t st) {
  if (nout <= 0) return hipSuccess;
  if (q < 1 || w <= q) return hipErrorInvalidValue;
  const int64_t F = w / q;
  if (F < 2 || F > kArgColsMaxF || (F + 1) * q < w) return hipErrorInvalidValue;
  int B = 1;
  while (2 * B <= F) B *= 2;
  const int64_t rows = (nout + q - 1) / q;
  const int64_t strips = (q + 63) / 64;
  // about 4096 wavefronts; a band's locations relative to its first row
  // stay below 2^31
  const int64_t bands0 = std::max<int64_t>(1, 4096 / strips);
  int64_t TR = (rows + bands0 - 1) / bands0;
  TR = std::max<int64_t>(TR, 4 * B);
  TR = std::min<int64_t>(TR, ((int64_t(1) << 31) - 1) / q - F - 1);
  if (TR < 1) return hipErrorInvalidValue;
  TR = std::min<int64_t>(TR, rows);
  const int64_t bands = (rows + TR - 1) / TR;
  const int64_t ntiles = strips * bands;
  const int64_t grid = (ntiles + 7) / 8 * 8;
  if (grid > 0x7fffffff) return hipErrorInvalidValue;
  auto go = [&](auto* p) -> hipError_t {
    using T = std::remove_pointer_t<decltype(p)>;
    ArgColsArgs<T> a;
    a.vx = (const T*)vx;
    a.ix = ix;
    a.vn = (const T*)vn;
    a.in = in;
    a.nlv = nlv;
    a.q = q;
    a.w = w;
    a.nout = nout;
    a.F = (int)F;
    a.ox = (T*)ox;
    a.jx = jx;
    a.on = (T*)on;
    a.jn = jn;
    a.rows = rows;
    a.strips = (int)strips;
    a.TR = (int)TR;
    a.ntiles = ntiles;
    const dim3 g((unsigned)grid), blk(64);
    switch (B) {
      case 1: hipLaunchKernelGGL((k_argcols<T, 1>), g, blk, 0, st, a); break;
      case 2: hipLaunchKernelGGL((k_argcols<T, 2>), g, blk, 0, st, a); break;
      case 4: hipLaunchKernelGGL((k_argcols<T, 4>), g, blk, 0, st, a); break;
      case 8: hipLaunchKernelGGL((k_argcols<T, 8>), g, blk, 0, st, a); break;
      default: hipLaunchKernelGGL((k_argcols<T, 16>), g, blk, 0, st, a); break;
    }
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
