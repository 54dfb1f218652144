// gfx950 batched centered envelopes of short series: the maximum and
// minimum over [i-r, i+r], truncated at the series ends, for every sample
// i (the lower/upper bounds used for time-warping searches, Section 1).
//
// One wavefront per series (env_short: n <= kEnvShortN, r <= kEnvShortR),
// in segments of 512 outputs.  Each segment filters its 512 + 2r inputs
// with window 2r+1 by the row filter of the fused 2-D pass.  A position
// before the series start reads sample 0 and one past its end reads sample
// n-1: both lie in every truncated window that reaches past that end, so
// the clamped windows have exactly the truncated windows' max and min --
// no identity padding, no separate end passes.
#include "mm_f2d.hpp"

namespace mm {

template <class T>
__global__ __launch_bounds__(256) void k_env_short(const T* in, const int64_t* off, const int64_t* radii, int64_t S,
                                                   T* up, T* lo) {
  constexpr int V = 8, W = 64 * V;
  __shared__ T hpx[4][lds_len<T>(2 * W)], hpn[4][lds_len<T>(2 * W)];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t k = (int64_t)blockIdx.x * 4 + wv;  // one series per wavefront (no block barriers)
  if (k >= S) return;
  const int64_t s0 = off[k], n = off[k + 1] - s0, r = radii[k];
  if (!env_short(n, r)) return;
  const int wc = (int)(2 * r + 1);
  const int lgBh = 31 - __builtin_clz((unsigned)min(wc, 16 * V));
  const int Bh = 1 << lgBh;
  const int mh = Bh > V ? Bh / V : 1;
  const int lig = lane & (mh - 1);
  const int kmax = max(0, (wc + Bh - 2) / Bh - 1);
  const T* a = in + s0;
  T* const bx = hpx[wv];  // the row buffer also stages loads and stores
  T* const bn = hpn[wv];
  const int np = W + wc - 1;  // inputs of a segment, <= 2W
  for (int64_t c0 = 0; c0 < n; c0 += W) {
    // lane-consecutive (coalesced) loads into LDS, then V consecutive
    // positions per lane (series start anywhere: no vector alignment); all
    // loads are issued before the first is used (a loop storing each load
    // as it arrives ran 20% slower)
    T ld[2 * V];
#pragma unroll
    for (int u = 0; u < 2 * V; ++u) {
      const int p = u * 64 + lane;
      ld[u] = gload(a + min(max(c0 - r + (p < np ? p : 0), (int64_t)0), n - 1));
    }
#pragma unroll
    for (int u = 0; u < 2 * V; ++u)
      if (u * 64 + lane < np) bx[lds_idx<T>(u * 64 + lane)] = ld[u];
    f2_wave_sync();
    T x[V], h[V], rx[V], rn[V];
#pragma unroll
    for (int i = 0; i < V; ++i) {
      x[i] = bx[lds_idx<T>(lane * V + i)];
      h[i] = bx[lds_idx<T>(W + lane * V + i)];  // past np: unused positions
    }
    f2_wave_sync();
    f2_row_filter<T, V, 0, true, true>(x, h, wc, lgBh, mh, lig, kmax, bx, bn, rx, rn);
    f2_wave_sync();
#pragma unroll
    for (int i = 0; i < V; ++i) {
      bx[lds_idx<T>(lane * V + i)] = rx[i];
      bn[lds_idx<T>(lane * V + i)] = rn[i];
    }
    f2_wave_sync();
    for (int p = lane; p < W; p += 64) {
      const int64_t o = c0 + p;
      if (o < n) {
        gstore(up + s0 + o, bx[lds_idx<T>(p)]);
        gstore(lo + s0 + o, bn[lds_idx<T>(p)]);
      }
    }
    f2_wave_sync();  // the buffer is rewritten by the next segment
  }
}

hipError_t launch_env_short(int dtype, const void* in, const int64_t* off, const int64_t* radii, int64_t S, void* up,
                            void* lo, hipStream_t st) {
  if (S <= 0) return hipSuccess;
  const int64_t g = (S + 3) / 4;
  if (g > 0x7fffffff) return hipErrorInvalidValue;
  auto go = [&](auto* p) -> hipError_t {
    using T = std::remove_pointer_t<decltype(p)>;
    hipLaunchKernelGGL(k_env_short<T>, dim3((unsigned)g), dim3(256), 0, st, (const T*)in, off, radii, S, (T*)up,
                       (T*)lo);
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
