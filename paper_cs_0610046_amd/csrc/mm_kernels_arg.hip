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
