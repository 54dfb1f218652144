// gfx950 column pass of the 2-D filter (Section 1: the 1-D filter applied to
// rows, then to columns).  The row pass is the 1-D kernels' "rows" job; this
// kernel filters the columns of the row-filtered max image (maxima) and min
// image (minima).
//
// One wavefront owns 64 adjacent columns and one block of w_r output rows
// (van Herk / Gil-Werman with blocks of exactly w_r rows): walking its own
// block bottom-up it keeps the suffix maxima/minima of every row in LDS; then
// walking the next block top-down it keeps the running prefix and emits
//     out[r0+i] = max(SUF[r0+i], PRE[r0+w_r-1+i]).
// Each row access is 64 consecutive elements of one image row (coalesced);
// loads are issued in batches of 8 rows to keep them in flight.
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

// The same column pass with each column's block suffixes in registers (4-
// and 2-byte data, w_rows <= 64): two 32-slot vectors per image, indexed by
// a wavefront-uniform slot number (indirect register addressing), so no
// LDS: 183 VGPRs, two wavefronts per SIMD instead of the five per CU that
// 32 KiB of LDS per wavefront allowed at w_rows = 63.
typedef unsigned int cr_u32x32 __attribute__((ext_vector_type(32)));
struct CrRing {
  cr_u32x32 a, b;
};
template <class T> __device__ __forceinline__ uint32_t cr_bits(T v) {
  if constexpr (sizeof(T) == 4) return __builtin_bit_cast(uint32_t, v);
  else return (uint32_t)__builtin_bit_cast(uint16_t, v);
}
template <class T> __device__ __forceinline__ T cr_val(uint32_t b) {
  if constexpr (sizeof(T) == 4) return __builtin_bit_cast(T, b);
  else return __builtin_bit_cast(T, (uint16_t)b);
}
__device__ __forceinline__ void cr_set(CrRing& r, int i, uint32_t v) {
  i = __builtin_amdgcn_readfirstlane(i);
  if (i < 32) r.a[i] = v;
  else r.b[i - 32] = v;
}
__device__ __forceinline__ uint32_t cr_get(const CrRing& r, int i) {
  i = __builtin_amdgcn_readfirstlane(i);
  return i < 32 ? r.a[i] : r.b[i - 32];
}

template <class T>
__global__ __launch_bounds__(64) void k_cols_reg(const T* __restrict__ M, const T* __restrict__ N, int64_t ld_t,
                                                 int64_t rows, int64_t oc, int64_t w, T* __restrict__ omax,
                                                 T* __restrict__ omin, int64_t ld_out) {
  static_assert(sizeof(T) <= 4, "32-bit register slots");
  const int lane = threadIdx.x;
  const bool hx = M != nullptr, hn = N != nullptr;
  const int64_t c = (int64_t)blockIdx.x * 64 + lane;
  const bool act = c < oc;
  const int64_t cc = act ? c : 0;
  const int64_t orows = rows - w + 1;
  const int64_t r0 = (int64_t)blockIdx.y * w;  // first output row of the block
  if (r0 >= orows) return;
  const int64_t nb = min(w, orows - r0);  // outputs of this block
  CrRing Sx, Sn;
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
        cr_set(Sx, (int)i, cr_bits(sx));
        cr_set(Sn, (int)i, cr_bits(sn));
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
          if (hx) omax[(r0 + i) * ld_out + c] = vmax(cr_val<T>(cr_get(Sx, (int)i)), px);
          if (hn) omin[(r0 + i) * ld_out + c] = vmin(cr_val<T>(cr_get(Sn, (int)i)), pn);
        }
      }
    }
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
    if constexpr (sizeof(T) <= 4) {
      // from w_rows 49 on (MI355X, 8192^2 float32 rows-then-columns: w = 63
      // 0.55 against 0.64 ms; w = 48 equal, w <= 40 the LDS version ahead
      // by 5-10%); MAXMIN_COLS_LDS=1 keeps the LDS version (experiments)
      if (wr > 48 && wr <= 64 && !getenv("MAXMIN_COLS_LDS")) {
        hipLaunchKernelGGL((k_cols_reg<T>), grid, dim3(64), 0, st, (const T*)tmax, (const T*)tmin, ld_t, rows, oc,
                           wr, (T*)d_max, (T*)d_min, ld_out);
        return hipGetLastError();
      }
    }
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
