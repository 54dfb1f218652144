// Device-side building blocks shared by the gfx950 max-min kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mm {

// ---------------------------------------------------------------- values
// Identity elements: lo() for a running maximum, hi() for a running minimum.
template <class T> struct Lim;
template <> struct Lim<float> {
  __device__ static float lo() { return -__builtin_huge_valf(); }
  __device__ static float hi() { return __builtin_huge_valf(); }
};
template <> struct Lim<double> {
  __device__ static double lo() { return -__builtin_huge_val(); }
  __device__ static double hi() { return __builtin_huge_val(); }
};
template <> struct Lim<int32_t> {
  __device__ static int32_t lo() { return INT32_MIN; }
  __device__ static int32_t hi() { return INT32_MAX; }
};
template <> struct Lim<uint16_t> {
  __device__ static uint16_t lo() { return 0; }
  __device__ static uint16_t hi() { return 0xFFFF; }
};

// Selection only: compare, then pick one operand's bits unchanged.
template <class T> __device__ __forceinline__ T vmax(T a, T b) { return a > b ? a : b; }
template <class T> __device__ __forceinline__ T vmin(T a, T b) { return a < b ? a : b; }
// hmax / hmin: the same selection through the hardware max/min instruction
// for floating types.  For the inputs the library accepts (NaN-free; +-inf,
// subnormals and -0.0 allowed) v_max / v_min return one operand's bits
// unchanged, exactly as the compare-select does: the larger (smaller)
// value, and equal values other than +0.0 / -0.0 have equal bits (a window
// holding both zeros may return either, as the ABI states); denormals pass
// through (the kernels run with FP32/FP64 denormals preserved).  Written as one instruction each: through the
// compiler's maxnum the same instruction comes with a canonicalising max of
// every loaded or shuffled operand, which cost more than it saved in the
// tile kernel.  On MI355X (n = 2^28 float32) this took the tile kernel from
// 0.69-0.73 ms to 0.65-0.66 ms and the chunk kernel down by 2-5%.
template <class T> __device__ __forceinline__ T hmax(T a, T b) { return vmax(a, b); }
template <class T> __device__ __forceinline__ T hmin(T a, T b) { return vmin(a, b); }
template <> __device__ __forceinline__ float hmax<float>(float a, float b) {
  float r;
  asm("v_max_f32 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
  return r;
}
template <> __device__ __forceinline__ float hmin<float>(float a, float b) {
  float r;
  asm("v_min_f32 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
  return r;
}
template <> __device__ __forceinline__ double hmax<double>(double a, double b) {
  double r;
  asm("v_max_f64 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
  return r;
}
template <> __device__ __forceinline__ double hmin<double>(double a, double b) {
  double r;
  asm("v_min_f64 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
  return r;
}
template <bool HW, class T> __device__ __forceinline__ T smax(T a, T b) {
  if constexpr (HW) return hmax(a, b);
  else return vmax(a, b);
}
template <bool HW, class T> __device__ __forceinline__ T smin(T a, T b) {
  if constexpr (HW) return hmin(a, b);
  else return vmin(a, b);
}

// A value with its location (relative to a known origin), for the arg
// max/min filter.  Selection orders by value, then prefers the smaller
// location, so every combine returns the leftmost extremum whatever the
// operand order: the result is the same for any grouping of the scans.
template <class T> struct Loc {
  T v;
  int i;
};
template <class T> __device__ __forceinline__ Loc<T> vmax(Loc<T> a, Loc<T> b) {
  return (a.v > b.v || (a.v == b.v && a.i < b.i)) ? a : b;
}
template <class T> __device__ __forceinline__ Loc<T> vmin(Loc<T> a, Loc<T> b) {
  return (a.v < b.v || (a.v == b.v && a.i < b.i)) ? a : b;
}
// an element of the tile kernel: the value, or the value and its location
template <class T, bool ARG> struct ElemOf { typedef T type; };
template <class T> struct ElemOf<T, true> { typedef Loc<T> type; };
template <class T> __device__ __forceinline__ T elem(T v, int, T*) { return v; }
template <class T> __device__ __forceinline__ Loc<T> elem(T v, int i, Loc<T>*) { return Loc<T>{v, i}; }
template <class T> __device__ __forceinline__ T value_of(T e) { return e; }
template <class T> __device__ __forceinline__ T value_of(Loc<T> e) { return e.v; }

// ---------------------------------------------------------------- LDS layout
// One pad element per 128 bytes: a thread reading V consecutive elements and
// a wave writing lane-consecutive elements both stay clear of bank conflicts.
template <class T> struct Pad {
  static constexpr int sh = sizeof(T) == 16 ? 3 : (sizeof(T) == 8 ? 4 : (sizeof(T) == 4 ? 5 : 6));
};
template <class T> __host__ __device__ constexpr int lds_idx(int i) { return i + (i >> Pad<T>::sh); }
template <class T> __host__ __device__ constexpr int lds_len(int n) { return n + (n >> Pad<T>::sh) + 1; }

// ---------------------------------------------------------------- shuffles
template <class T> __device__ __forceinline__ T shup(T v, unsigned d, int width) {
  return __shfl_up(v, d, width);
}
template <> __device__ __forceinline__ uint16_t shup<uint16_t>(uint16_t v, unsigned d, int width) {
  return (uint16_t)__shfl_up((unsigned)v, d, width);
}
template <class T> __device__ __forceinline__ T shdn(T v, unsigned d, int width) {
  return __shfl_down(v, d, width);
}
template <> __device__ __forceinline__ uint16_t shdn<uint16_t>(uint16_t v, unsigned d, int width) {
  return (uint16_t)__shfl_down((unsigned)v, d, width);
}
template <class T> __device__ __forceinline__ Loc<T> shup(Loc<T> v, unsigned d, int width) {
  return Loc<T>{shup(v.v, d, width), __shfl_up(v.i, d, width)};
}
template <class T> __device__ __forceinline__ Loc<T> shdn(Loc<T> v, unsigned d, int width) {
  return Loc<T>{shdn(v.v, d, width), __shfl_down(v.i, d, width)};
}

// ---------------------------------------------------------------- DPP
// Cross-lane moves without LDS addresses: update_dpp(old, src, ctrl) gives
// each lane src from the lane `ctrl` names, or `old` where that lane lies
// outside the 16-lane row (bound_ctrl off).  Wider types move as 32-bit
// halves; 16-bit values travel zero-extended.
template <int CTRL> __device__ __forceinline__ uint32_t dpp32(uint32_t old, uint32_t src) {
  return (uint32_t)__builtin_amdgcn_update_dpp((int)old, (int)src, CTRL, 0xf, 0xf, false);
}
template <int CTRL, class T> __device__ __forceinline__ T dpp(T old, T src) {
  if constexpr (sizeof(T) == 8) {
    const uint64_t o = __builtin_bit_cast(uint64_t, old), v = __builtin_bit_cast(uint64_t, src);
    const uint32_t lo = dpp32<CTRL>((uint32_t)o, (uint32_t)v);
    const uint32_t hi = dpp32<CTRL>((uint32_t)(o >> 32), (uint32_t)(v >> 32));
    return __builtin_bit_cast(T, ((uint64_t)hi << 32) | lo);
  } else if constexpr (sizeof(T) == 4) {
    return __builtin_bit_cast(T, dpp32<CTRL>(__builtin_bit_cast(uint32_t, old), __builtin_bit_cast(uint32_t, src)));
  } else {
    return (T)dpp32<CTRL>((uint32_t)__builtin_bit_cast(uint16_t, old), (uint32_t)__builtin_bit_cast(uint16_t, src));
  }
}
template <class T> __device__ __forceinline__ T readlane(T v, int lane) {
  if constexpr (sizeof(T) == 8) {
    const uint64_t b = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, lane);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), lane);
    return __builtin_bit_cast(T, ((uint64_t)hi << 32) | lo);
  } else if constexpr (sizeof(T) == 4) {
    return __builtin_bit_cast(T, (uint32_t)__builtin_amdgcn_readlane((int)__builtin_bit_cast(uint32_t, v), lane));
  } else {
    return (T)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)__builtin_bit_cast(uint16_t, v), lane);
  }
}

// Inclusive prefix (in lane order) of max and min over the 64-lane wave.
// HW: select with hmax / hmin instead of vmax / vmin.
template <class T, bool HW = false> __device__ __forceinline__ void wave_prefix2(T& x, T& n) {
  const T lo = Lim<T>::lo(), hi = Lim<T>::hi();
  x = smax<HW>(x, dpp<0x111>(lo, x)); n = smin<HW>(n, dpp<0x111>(hi, n));  // row_shr:1
  x = smax<HW>(x, dpp<0x112>(lo, x)); n = smin<HW>(n, dpp<0x112>(hi, n));  // row_shr:2
  x = smax<HW>(x, dpp<0x114>(lo, x)); n = smin<HW>(n, dpp<0x114>(hi, n));  // row_shr:4
  x = smax<HW>(x, dpp<0x118>(lo, x)); n = smin<HW>(n, dpp<0x118>(hi, n));  // row_shr:8
  const int row = (threadIdx.x & 63) >> 4;
  const T x0 = readlane(x, 15), x1 = readlane(x, 31), x2 = readlane(x, 47);
  const T n0 = readlane(n, 15), n1 = readlane(n, 31), n2 = readlane(n, 47);
  if (row >= 1) { x = smax<HW>(x, x0); n = smin<HW>(n, n0); }
  if (row >= 2) { x = smax<HW>(x, x1); n = smin<HW>(n, n1); }
  if (row >= 3) { x = smax<HW>(x, x2); n = smin<HW>(n, n2); }
}

// Inclusive suffix (from the last lane down) of max and min over the wave.
template <class T, bool HW = false> __device__ __forceinline__ void wave_suffix2(T& x, T& n) {
  const T lo = Lim<T>::lo(), hi = Lim<T>::hi();
  x = smax<HW>(x, dpp<0x101>(lo, x)); n = smin<HW>(n, dpp<0x101>(hi, n));  // row_shl:1
  x = smax<HW>(x, dpp<0x102>(lo, x)); n = smin<HW>(n, dpp<0x102>(hi, n));  // row_shl:2
  x = smax<HW>(x, dpp<0x104>(lo, x)); n = smin<HW>(n, dpp<0x104>(hi, n));  // row_shl:4
  x = smax<HW>(x, dpp<0x108>(lo, x)); n = smin<HW>(n, dpp<0x108>(hi, n));  // row_shl:8
  const int row = (threadIdx.x & 63) >> 4;
  const T x1 = readlane(x, 16), x2 = readlane(x, 32), x3 = readlane(x, 48);
  const T n1 = readlane(n, 16), n2 = readlane(n, 32), n3 = readlane(n, 48);
  if (row <= 2) { x = smax<HW>(x, x3); n = smin<HW>(n, n3); }
  if (row <= 1) { x = smax<HW>(x, x2); n = smin<HW>(n, n2); }
  if (row <= 0) { x = smax<HW>(x, x1); n = smin<HW>(n, n1); }
}

// Inclusive scans of (max, min) over aligned groups of m lanes (m a power of
// two in 2..64, the same in every lane; lig = lane & (m-1)): prefix in lane
// order, or suffix.  DPP row shifts inside the 16-lane rows (a lane whose
// source lies in another group keeps its value), readlane across rows.
template <class T, bool HW>
__device__ __forceinline__ void seg_prefix2(T& x, T& n, int m, int lig) {
  const T lo = Lim<T>::lo(), hi = Lim<T>::hi();
  T a = dpp<0x111>(lo, x), b = dpp<0x111>(hi, n);  // row_shr:1
  x = lig >= 1 ? smax<HW>(x, a) : x;
  n = lig >= 1 ? smin<HW>(n, b) : n;
  if (m > 2) {
    a = dpp<0x112>(lo, x), b = dpp<0x112>(hi, n);  // row_shr:2
    x = lig >= 2 ? smax<HW>(x, a) : x;
    n = lig >= 2 ? smin<HW>(n, b) : n;
  }
  if (m > 4) {
    a = dpp<0x114>(lo, x), b = dpp<0x114>(hi, n);  // row_shr:4
    x = lig >= 4 ? smax<HW>(x, a) : x;
    n = lig >= 4 ? smin<HW>(n, b) : n;
  }
  if (m > 8) {
    a = dpp<0x118>(lo, x), b = dpp<0x118>(hi, n);  // row_shr:8
    x = lig >= 8 ? smax<HW>(x, a) : x;
    n = lig >= 8 ? smin<HW>(n, b) : n;
  }
  if (m > 16) {
    const int row = (threadIdx.x & 63) >> 4;
    const T x0 = readlane(x, 15), x1 = readlane(x, 31), x2 = readlane(x, 47);
    const T n0 = readlane(n, 15), n1 = readlane(n, 31), n2 = readlane(n, 47);
    if (m == 32) {
      // groups: rows 0-1 and rows 2-3
      if (row == 1) { x = smax<HW>(x, x0); n = smin<HW>(n, n0); }
      if (row == 3) { x = smax<HW>(x, x2); n = smin<HW>(n, n2); }
    } else {
      if (row >= 1) { x = smax<HW>(x, x0); n = smin<HW>(n, n0); }
      if (row >= 2) { x = smax<HW>(x, x1); n = smin<HW>(n, n1); }
      if (row >= 3) { x = smax<HW>(x, x2); n = smin<HW>(n, n2); }
    }
  }
}
template <class T, bool HW>
__device__ __forceinline__ void seg_suffix2(T& x, T& n, int m, int lig) {
  const T lo = Lim<T>::lo(), hi = Lim<T>::hi();
  T a = dpp<0x101>(lo, x), b = dpp<0x101>(hi, n);  // row_shl:1
  x = lig + 1 < m ? smax<HW>(x, a) : x;
  n = lig + 1 < m ? smin<HW>(n, b) : n;
  if (m > 2) {
    a = dpp<0x102>(lo, x), b = dpp<0x102>(hi, n);  // row_shl:2
    x = lig + 2 < m ? smax<HW>(x, a) : x;
    n = lig + 2 < m ? smin<HW>(n, b) : n;
  }
  if (m > 4) {
    a = dpp<0x104>(lo, x), b = dpp<0x104>(hi, n);  // row_shl:4
    x = lig + 4 < m ? smax<HW>(x, a) : x;
    n = lig + 4 < m ? smin<HW>(n, b) : n;
  }
  if (m > 8) {
    a = dpp<0x108>(lo, x), b = dpp<0x108>(hi, n);  // row_shl:8
    x = lig + 8 < m ? smax<HW>(x, a) : x;
    n = lig + 8 < m ? smin<HW>(n, b) : n;
  }
  if (m > 16) {
    const int row = (threadIdx.x & 63) >> 4;
    const T x1 = readlane(x, 16), x2 = readlane(x, 32), x3 = readlane(x, 48);
    const T n1 = readlane(n, 16), n2 = readlane(n, 32), n3 = readlane(n, 48);
    if (m == 32) {
      if (row == 0) { x = smax<HW>(x, x1); n = smin<HW>(n, n1); }
      if (row == 2) { x = smax<HW>(x, x3); n = smin<HW>(n, n3); }
    } else {
      if (row <= 2) { x = smax<HW>(x, x3); n = smin<HW>(n, n3); }
      if (row <= 1) { x = smax<HW>(x, x2); n = smin<HW>(n, n2); }
      if (row <= 0) { x = smax<HW>(x, x1); n = smin<HW>(n, n1); }
    }
  }
}

// ---------------------------------------------------------------- series
// One series of the 1-D filter.  Its n elements are the concatenation of two
// segments: element i is a[i] for i < na, else b[i - na].  A plain call has
// na = n; a stream push puts its carried samples in `a` and the new chunk in
// `b`.  Outputs: n_out = max(0, n - w + 1) maxima and minima.  If `carry` is
// non-null the last min(n, w-1) inputs are also copied there (the next
// push's carry).
template <class T> struct Series {
  const T* a;
  const T* b;
  int64_t na;
  int64_t n;
  int64_t w;
  T* omax;
  T* omin;
  T* carry;
};

// Series data always lives in global memory: access it through the global
// address space so the compiler emits global_* (not flat_*) instructions,
// which neither take the LDS-aperture check nor count against lgkmcnt.
template <class T> __device__ __forceinline__ T gload(const T* p) {
  return *(const __attribute__((address_space(1))) T*)p;
}
template <class T> __device__ __forceinline__ void gstore(T* p, T v) {
  *(__attribute__((address_space(1))) T*)p = v;
}
// Streaming store (nontemporal hint).  On MI355X it sped up the chunk
// kernel's staged 16-byte output stores by ~3% and slowed the tile kernel's.
template <class T> __device__ __forceinline__ void gstore_nt(T* p, T v) {
  __builtin_nontemporal_store(v, (__attribute__((address_space(1))) T*)p);
}

template <class T> __device__ __forceinline__ T src_at(const Series<T>& s, int64_t i) {
  return i < s.na ? gload(s.a + i) : gload(s.b + (i - s.na));
}

// ---------------------------------------------------------------- atomics
__device__ __forceinline__ void st_agent(uint64_t* p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t ld_agent(const uint64_t* p) {
  return __hip_atomic_load(const_cast<uint64_t*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t ld_agent32(const uint32_t* p) {
  return __hip_atomic_load(const_cast<uint32_t*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_agent32(uint32_t* p, uint32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t add_agent32(uint32_t* p, uint32_t v) {
  return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <class T> __device__ __forceinline__ uint64_t to_bits(T v) {
  if constexpr (sizeof(T) == 8) return __builtin_bit_cast(uint64_t, v);
  else if constexpr (sizeof(T) == 4) return (uint64_t)__builtin_bit_cast(uint32_t, v);
  else return (uint64_t)__builtin_bit_cast(uint16_t, v);
}
template <class T> __device__ __forceinline__ T from_bits(uint64_t b) {
  if constexpr (sizeof(T) == 8) return __builtin_bit_cast(T, b);
  else if constexpr (sizeof(T) == 4) return __builtin_bit_cast(T, (uint32_t)b);
  else return __builtin_bit_cast(T, (uint16_t)b);
}

// Per-launch control words in device memory (one set per HIP stream).
constexpr int kMaxRanges = 32;
struct Ctl {
  uint32_t ticket;  // next chunk tile to hand out (in-order tickets)
  uint32_t done;    // workgroups that have left the persistent loop
  uint32_t epoch;   // tags this launch's published aggregates
  uint32_t err;     // non-zero: a look-back wait gave up (never expected)
  uint32_t pad[28];
  uint32_t tick[kMaxRanges][32];  // per-range tickets, one 128-byte line each
};

// Look-back records of the chunk strategy: 2^lg records of 4 words each.
struct FlagRing {
  uint64_t* f;
  uint32_t lg;
};

// One launch of a 1-D kernel (see JobMode in the kernel source).
template <class T> struct Job {
  int mode;
  Series<T> one;          // single series
  int64_t ntiles;         // single series and rows: total tiles of the launch
  const Series<T>* descs; // described series
  const int64_t* pre;     // S+1 tile prefix sums (entry S = total)
  int64_t S;
  const T* in;            // rows: series k = in[k*ld_in .. k*ld_in + n)
  int64_t ld_in;
  int64_t n;
  int64_t w;
  T* omax;                // rows: outputs of series k at omax/omin + k*ld_out
  T* omin;
  int64_t ld_out;
  int64_t tpr;            // rows: tiles per row
  int64_t run;            // tile strategy: windows per run (a multiple of the sub-tile)
  int64_t* amax;          // arg filter (single series, tile strategy): locations of the
  int64_t* amin;          //   leftmost max / min of every window, else null
  int ranges;             // chunk strategy, single series: ticket ranges (0: one counter)
  FlagRing ring;          // chunk strategy only
  Ctl* ctl;
};

}  // namespace mm
