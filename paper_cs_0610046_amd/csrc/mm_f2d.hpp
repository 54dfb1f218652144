// gfx950 fused 2-D filter (Section 1: the 1-D filter on rows, then on
// columns, here in one pass) -- kernel and launcher templates, instantiated
// per output set in mm_kernels_2d*.hip.
#pragma once

#include <algorithm>
#include <type_traits>

#include "mm_launch.hpp"

namespace mm {

// One pass over the image for w_rows <= 64 and w_cols <= 64 * V + 1: a
// wavefront owns a strip of 64*V output columns (two such half-strips for
// 16-bit data, packed) and a band of output rows and streams down the
// band's input rows.  Each row is filtered along the
// row in registers (blocks of Bh columns, PRE through an LDS row buffer,
// SUF in registers: the 1-D tile scheme on one row of 64*V + w_cols - 1
// inputs); the row results then feed a column filter with blocks of B
// rows, kept per lane in an LDS ring of 2B rows: a block's raw values turn
// into its suffixes when the next block starts, and the output of the
// window that ends at the current row is
//     max(SUF[first row], aggregate of the block between, running PRE).
// Every lane owns its columns of the ring, so only the row buffer needs
// barriers.  The max and min images never leave the chip: HBM traffic is
// the input (plus the halo rows and columns) and the outputs.
typedef unsigned int f2_u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int f2_u32x2 __attribute__((ext_vector_type(2)));

// 16-bit images run packed: a lane value holds the same position of two
// half-strips 64 V columns apart (low half: the left one), so that every
// selection is one v_pk_max_u16 / v_pk_min_u16 for two pixels and the
// kernel's logic is unchanged.  F2Store gives the image element type.
struct P16 {
  uint32_t v;
};
template <> struct Lim<P16> {
  __device__ static P16 lo() { return P16{0u}; }
  __device__ static P16 hi() { return P16{0xFFFFFFFFu}; }
};
template <> __device__ __forceinline__ P16 hmax<P16>(P16 a, P16 b) {
  P16 r;
  asm("v_pk_max_u16 %0, %1, %2" : "=v"(r.v) : "v"(a.v), "v"(b.v));
  return r;
}
template <> __device__ __forceinline__ P16 hmin<P16>(P16 a, P16 b) {
  P16 r;
  asm("v_pk_min_u16 %0, %1, %2" : "=v"(r.v) : "v"(a.v), "v"(b.v));
  return r;
}
template <class T> struct F2Store {
  typedef T S;
  static constexpr int halves = 1;
};
template <> struct F2Store<P16> {
  typedef uint16_t S;
  static constexpr int halves = 2;
};

template <class T> struct F2dArgs {
  const T* in;
  const T* in2;  // column-only mode: the row-filtered min image (in: the max image)
  int64_t ld_in, rows, cols;
  int wr, wc;
  T* omax;
  T* omin;
  int64_t ld_out;
  int strips, TR;
  int64_t ntiles;
};

// V consecutive elements at p.  Stores take the widest access (16, 8 or 4
// bytes) that p's alignment allows; lane offsets are multiples of V * s, so
// every lane of a wavefront takes the same branch for a given row.
template <class T, int V, bool VIN> __device__ __forceinline__ void f2_load(const T* p, T (&x)[V]) {
  // VIN: the launcher checked that every row start is aligned to the
  // access width (min(16, V * s) bytes); a branch on the address here would
  // make the compiler wait for each load where the branches join
  constexpr int NB = V * (int)sizeof(T);
  if constexpr (VIN && NB % 16 == 0) {
#pragma unroll
    for (int k = 0; k < NB / 16; ++k) {
      const f2_u32x4 u = gload((const f2_u32x4*)p + k);
      __builtin_memcpy((char*)x + 16 * k, &u, 16);
    }
  } else if constexpr (VIN && NB == 8) {
    const f2_u32x2 u = gload((const f2_u32x2*)p);
    __builtin_memcpy(x, &u, 8);
  } else if constexpr (VIN && NB == 4 && sizeof(T) < 4) {
    const unsigned u = gload((const unsigned*)p);
    __builtin_memcpy(x, &u, 4);
  } else {
#pragma unroll
    for (int i = 0; i < V; ++i) x[i] = gload(p + i);
  }
}
template <class T, int V> __device__ __forceinline__ void f2_store(T* p, const T (&x)[V]) {
  constexpr int NB = V * (int)sizeof(T);
  const uintptr_t ad = (uintptr_t)p;
  if constexpr (NB % 16 == 0) {
    if (ad % 16 == 0) {
#pragma unroll
      for (int k = 0; k < NB / 16; ++k) {
        f2_u32x4 u;
        __builtin_memcpy(&u, (const char*)x + 16 * k, 16);
        gstore((f2_u32x4*)p + k, u);
      }
      return;
    }
  }
  if constexpr (NB % 8 == 0) {
    if (ad % 8 == 0) {
#pragma unroll
      for (int k = 0; k < NB / 8; ++k) {
        f2_u32x2 u;
        __builtin_memcpy(&u, (const char*)x + 8 * k, 8);
        gstore((f2_u32x2*)p + k, u);
      }
      return;
    }
  }
  if constexpr (NB % 4 == 0 && sizeof(T) < 4) {
    if (ad % 4 == 0) {
#pragma unroll
      for (int k = 0; k < NB / 4; ++k) {
        unsigned u;
        __builtin_memcpy(&u, (const char*)x + 4 * k, 4);
        gstore((unsigned*)p + k, u);
      }
      return;
    }
  }
#pragma unroll
  for (int i = 0; i < V; ++i) gstore(p + i, x[i]);
}

// Loads of input row `row` for this lane: its V strip columns, and its V
// halo columns one strip width further (only the first wc-1 halo columns
// are read; the other lanes load lane 0's halo vector, one cache line).
// No lane-dependent branch: a branch whose sides write the load's
// registers would make every lane wait for the load; strips that reach the
// row end (a wave-uniform test) clamp each column instead.
// Column-only mode: the V columns of row `row` of the row-filtered images
// the call needs (max image into x, min image into h), clamped at the row
// end like the above.
// One input row of the lane in flight: for 4- and 8-byte data the lane
// values themselves (x: its V strip columns, h: V halo columns), for packed
// 16-bit data the raw dwords as loaded (a, b, c: half-strips A, B and B's
// halo; column-only mode: a, b the max image's halves, c, d the min
// image's), packed only when the row is used so that a load in flight is
// waited for just before its row.
template <class T, int V> struct F2Raw {
  T x[V], h[V];
};
template <int V> struct F2Raw<P16, V> {
  static constexpr int NW = (V + 1) / 2;
  uint32_t a[NW], b[NW], c[NW], d[NW];
};

// V 16-bit elements at p into (V + 1) / 2 dwords (element 2k low, 2k+1 high).
template <int V, bool VIN> __device__ __forceinline__ void f2_load16(const uint16_t* p, uint32_t (&w)[(V + 1) / 2]) {
  if constexpr (VIN && V == 8) {
    const f2_u32x4 u = gload((const f2_u32x4*)p);
    w[0] = u.x; w[1] = u.y; w[2] = u.z; w[3] = u.w;
  } else if constexpr (VIN && V == 4) {
    const f2_u32x2 u = gload((const f2_u32x2*)p);
    w[0] = u.x; w[1] = u.y;
  } else if constexpr (VIN && V == 2) {
    w[0] = gload((const uint32_t*)p);
  } else {
#pragma unroll
    for (int k = 0; k < (V + 1) / 2; ++k) {
      const uint32_t lo = gload(p + 2 * k);
      w[k] = 2 * k + 1 < V ? lo | ((uint32_t)gload(p + 2 * k + 1) << 16) : lo;
    }
  }
}
// the same, each column clamped to the row end (strips that reach it)
template <int V> __device__ __forceinline__ void f2_load16c(const uint16_t* rp, int64_t c, int64_t cols,
                                                          uint32_t (&w)[(V + 1) / 2]) {
#pragma unroll
  for (int k = 0; k < (V + 1) / 2; ++k) {
    const uint32_t lo = gload(rp + min(c + 2 * k, cols - 1));
    w[k] = 2 * k + 1 < V ? lo | ((uint32_t)gload(rp + min(c + 2 * k + 1, cols - 1)) << 16) : lo;
  }
}
// lane values from two halves' dwords: element i of half L low, of half H high
template <int V> __device__ __forceinline__ void f2_pack(const uint32_t (&L)[(V + 1) / 2],
                                                        const uint32_t (&H)[(V + 1) / 2], P16 (&v)[V]) {
#pragma unroll
  for (int i = 0; i < V; ++i)
    v[i].v = __builtin_amdgcn_perm(H[i / 2], L[i / 2], (i & 1) ? 0x07060302u : 0x05040100u);
}

template <class T, int V, bool VIN, int OUT>
__device__ __forceinline__ void f2_pair_issue(const F2dArgs<typename F2Store<T>::S>& a, int64_t row, int64_t c0,
                                              F2Raw<T, V>& r) {
  constexpr int W = 64 * V;
  const int lane = threadIdx.x & 63;
  const auto* px = a.in + row * a.ld_in;
  const auto* pn = a.in2 + row * a.ld_in;
  const int64_t cm = c0 + lane * V;
  if constexpr (F2Store<T>::halves == 2) {
    if (c0 + 2 * W <= a.cols) {
      if constexpr ((OUT & 1) != 0) {
        f2_load16<V, VIN>(px + cm, r.a);
        f2_load16<V, VIN>(px + cm + W, r.b);
      }
      if constexpr ((OUT & 2) != 0) {
        f2_load16<V, VIN>(pn + cm, r.c);
        f2_load16<V, VIN>(pn + cm + W, r.d);
      }
    } else {
      if constexpr ((OUT & 1) != 0) {
        f2_load16c<V>(px, cm, a.cols, r.a);
        f2_load16c<V>(px, cm + W, a.cols, r.b);
      }
      if constexpr ((OUT & 2) != 0) {
        f2_load16c<V>(pn, cm, a.cols, r.c);
        f2_load16c<V>(pn, cm + W, a.cols, r.d);
      }
    }
  } else if (c0 + W <= a.cols) {
    if constexpr ((OUT & 1) != 0) f2_load<T, V, VIN>(px + cm, r.x);
    if constexpr ((OUT & 2) != 0) f2_load<T, V, VIN>(pn + cm, r.h);
  } else {
#pragma unroll
    for (int i = 0; i < V; ++i) {
      if constexpr ((OUT & 1) != 0) r.x[i] = gload(px + min(cm + i, a.cols - 1));
      if constexpr ((OUT & 2) != 0) r.h[i] = gload(pn + min(cm + i, a.cols - 1));
    }
  }
}
template <class T, int V, int OUT>
__device__ __forceinline__ void f2_pair_take(const F2Raw<T, V>& r, T (&x)[V], T (&h)[V]) {
  if constexpr (F2Store<T>::halves == 2) {
    if constexpr ((OUT & 1) != 0) f2_pack<V>(r.a, r.b, x);
    if constexpr ((OUT & 2) != 0) f2_pack<V>(r.c, r.d, h);
  } else {
#pragma unroll
    for (int i = 0; i < V; ++i) {
      x[i] = r.x[i];
      h[i] = r.h[i];
    }
  }
}

template <class T, int V, bool VIN>
__device__ __forceinline__ void f2_row_issue(const F2dArgs<typename F2Store<T>::S>& a, int64_t row, int64_t c0,
                                             F2Raw<T, V>& r) {
  constexpr int W = 64 * V;
  const int lane = threadIdx.x & 63;
  const auto* rp = a.in + row * a.ld_in;
  const int64_t cm = c0 + lane * V, hoff = lane * V < a.wc - 1 ? lane * V : 0;
  if constexpr (F2Store<T>::halves == 2) {
    // half-strips A = [c0, c0+W) and B = [c0+W, c0+2W); A's halo is B, B's
    // halo the first wc-1 columns of C = [c0+2W, ...)
    const int64_t cc = c0 + 2 * W + hoff;
    if (c0 + 3 * W <= a.cols) {
      f2_load16<V, VIN>(rp + cm, r.a);
      f2_load16<V, VIN>(rp + cm + W, r.b);
      f2_load16<V, VIN>(rp + cc, r.c);
    } else {
      f2_load16c<V>(rp, cm, a.cols, r.a);
      f2_load16c<V>(rp, cm + W, a.cols, r.b);
      f2_load16c<V>(rp, cc, a.cols, r.c);
    }
  } else {
    const int64_t chh = c0 + W + hoff;
    if (c0 + 2 * W <= a.cols) {
      f2_load<T, V, VIN>(rp + cm, r.x);
      f2_load<T, V, VIN>(rp + chh, r.h);
    } else {
#pragma unroll
      for (int i = 0; i < V; ++i) {
        r.x[i] = gload(rp + min(cm + i, a.cols - 1));
        r.h[i] = gload(rp + min(chh + i, a.cols - 1));
      }
    }
  }
}
template <class T, int V> __device__ __forceinline__ void f2_row_take(const F2Raw<T, V>& r, T (&x)[V], T (&h)[V]) {
  if constexpr (F2Store<T>::halves == 2) {
    f2_pack<V>(r.a, r.b, x);
    f2_pack<V>(r.b, r.c, h);
  } else {
#pragma unroll
    for (int i = 0; i < V; ++i) {
      x[i] = r.x[i];
      h[i] = r.h[i];
    }
  }
}

// The lane's V outputs of one output row: vector stores where all of them
// exist (each half-strip separately when packed), else one by one.
template <class T, int V>
__device__ __forceinline__ void f2_out_store(typename F2Store<T>::S* o, int64_t cm, int64_t oc, const T (&v)[V]) {
  using S = typename F2Store<T>::S;
  if constexpr (F2Store<T>::halves == 2) {
    constexpr int W = 64 * V;
    uint32_t lo[(V + 1) / 2], hi[(V + 1) / 2];  // half A's columns, half B's
#pragma unroll
    for (int k = 0; k < (V + 1) / 2; ++k) {
      const uint32_t u = v[2 * k].v, w = 2 * k + 1 < V ? v[2 * k + 1].v : 0u;
      lo[k] = __builtin_amdgcn_perm(w, u, 0x05040100u);
      hi[k] = __builtin_amdgcn_perm(w, u, 0x07060302u);
    }
    auto put = [&](int64_t c, const uint32_t (&d)[(V + 1) / 2]) {
      S* p = o + c;
      const uintptr_t ad = (uintptr_t)p;
      if (c + V <= oc && V >= 2 && ad % (2 * V) == 0) {
        if constexpr (V == 8) {
          gstore((f2_u32x4*)p, f2_u32x4{d[0], d[1], d[2], d[3]});
        } else if constexpr (V == 4) {
          gstore((f2_u32x2*)p, f2_u32x2{d[0], d[1]});
        } else if constexpr (V == 2) {
          gstore((uint32_t*)p, d[0]);
        }
      } else if (c + V <= oc && V >= 2 && ad % 4 == 0) {
#pragma unroll
        for (int k = 0; k < V / 2; ++k) gstore((uint32_t*)p + k, d[k]);
      } else {
#pragma unroll
        for (int i = 0; i < V; ++i)
          if (c + i < oc) gstore(p + i, (S)(d[i / 2] >> (16 * (i & 1))));
      }
    };
    put(cm, lo);
    put(cm + W, hi);
  } else {
    if (cm + V <= oc) {
      f2_store<T, V>(o + cm, v);
    } else {
#pragma unroll
      for (int i = 0; i < V; ++i)
        if (cm + i < oc) gstore(o + cm + i, v[i]);
    }
  }
}

// Inclusive scans of (max, min) over aligned groups of m lanes, m a power
// of two in 2..16 (inside one DPP row).  A step of distance d must not
// reach into the previous (next) group: that happens exactly where the
// SOURCE lane has lig >= m - d (lig < d), so the source is masked to the
// identity there and every lane combines unconditionally -- a select on
// the DPP source, which the compiler keeps as one v_cndmask (a select on
// the result it turns into exec-masked branches).
template <class T, int D> __device__ __forceinline__ void f2_pre_step(T& x, T& n, int m, int lig) {
  const bool k = lig >= m - D;
  x = hmax(x, dpp<0x110 + D>(Lim<T>::lo(), k ? Lim<T>::lo() : x));  // row_shr:D
  n = hmin(n, dpp<0x110 + D>(Lim<T>::hi(), k ? Lim<T>::hi() : n));
}
template <class T, int D> __device__ __forceinline__ void f2_suf_step(T& x, T& n, int lig) {
  const bool k = lig < D;
  x = hmax(x, dpp<0x100 + D>(Lim<T>::lo(), k ? Lim<T>::lo() : x));  // row_shl:D
  n = hmin(n, dpp<0x100 + D>(Lim<T>::hi(), k ? Lim<T>::hi() : n));
}
template <class T> __device__ __forceinline__ void f2_seg_pre(T& x, T& n, int m, int lig) {
  f2_pre_step<T, 1>(x, n, m, lig);
  if (m > 2) f2_pre_step<T, 2>(x, n, m, lig);
  if (m > 4) f2_pre_step<T, 4>(x, n, m, lig);
  if (m > 8) f2_pre_step<T, 8>(x, n, m, lig);
}
template <class T> __device__ __forceinline__ void f2_seg_suf(T& x, T& n, int m, int lig) {
  f2_suf_step<T, 1>(x, n, lig);
  if (m > 2) f2_suf_step<T, 2>(x, n, lig);
  if (m > 4) f2_suf_step<T, 4>(x, n, lig);
  if (m > 8) f2_suf_step<T, 8>(x, n, lig);
}

// The workgroup is one wavefront, whose LDS accesses execute in order: a
// wavefront-scope fence keeps the compiler from moving them across, and,
// unlike a workgroup barrier, does not wait for the row loads in flight.
__device__ __forceinline__ void f2_wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// One row filtered along the row: x holds this lane's V positions of a
// row segment, h its V positions one segment width (64 V) further (only
// positions < 64 V + wc - 1 are read); rx / rn get max / min over
// [p, p + wc - 1] for the lane's positions p.  Blocks of Bh = 2^lgBh <= 16 V
// positions, mh = max(1, Bh / V) lanes each (lig = lane & (mh - 1)); at
// most kmax whole blocks inside a window.  KM > 0: read a fixed KM of them
// (KM = 1 when wc <= 16 V, as then Bh > wc / 2; else 4), clamped, so that
// all the reads of a row go out together; KM = 0: a loop to kmax (fewer
// registers live: the one-output kernels and the envelopes keep it).  hpx / hpn: this wavefront's LDS row
// buffer of lds_len<T>(128 V) elements (only the side WX / WN is used).
// The caller orders the buffer's next reuse (f2_wave_sync).
template <class T, int V, int KM, bool WX, bool WN>
__device__ __forceinline__ void f2_row_filter(const T (&x)[V], const T (&h)[V], int wc, int lgBh, int mh, int lig,
                                              int kmax, T* hpx, T* hpn, T (&rx)[V], T (&rn)[V]) {
  constexpr int W = 64 * V;
  const int lane = threadIdx.x & 63;
  const int Bh = 1 << lgBh;
  T px[V], pn[V], qx[V], qn[V], sx[V], sn[V];
  px[0] = pn[0] = x[0];
  qx[0] = qn[0] = h[0];
#pragma unroll
  for (int i = 1; i < V; ++i) {
    // hmax / hmin are inline asm, which the compiler never moves into
    // a branch: take them unconditionally, then select (no branches)
    const bool st = ((lane * V + i) & (Bh - 1)) == 0;  // same phase in the halo (W % Bh == 0)
    const T ax = hmax(px[i - 1], x[i]), an = hmin(pn[i - 1], x[i]);
    const T bxx = hmax(qx[i - 1], h[i]), bnn = hmin(qn[i - 1], h[i]);
    px[i] = st ? x[i] : ax;
    pn[i] = st ? x[i] : an;
    qx[i] = st ? h[i] : bxx;
    qn[i] = st ? h[i] : bnn;
  }
  sx[V - 1] = sn[V - 1] = x[V - 1];
#pragma unroll
  for (int i = V - 2; i >= 0; --i) {
    const bool en = ((lane * V + i + 1) & (Bh - 1)) == 0;
    const T ax = hmax(sx[i + 1], x[i]), an = hmin(sn[i + 1], x[i]);
    sx[i] = en ? x[i] : ax;
    sn[i] = en ? x[i] : an;
  }
  if (mh > 1) {
    // lane totals scanned over the block's lanes; each lane then takes
    // the scan of the lane before (PRE) or after (SUF) it in its block
    T ix = px[V - 1], in = pn[V - 1], jx = qx[V - 1], jn = qn[V - 1], kx = sx[0], kn = sn[0];
    f2_seg_pre(ix, in, mh, lig);
    f2_seg_pre(jx, jn, mh, lig);
    f2_seg_suf(kx, kn, mh, lig);
    // (the source lane masked as in the scans: the last lane of a
    // group passes nothing on to the next, the first nothing back)
    const T lo = Lim<T>::lo(), hi = Lim<T>::hi();
    const bool lp = lig == mh - 1, ls = lig == 0;
    const T cx = dpp<0x111>(lo, lp ? lo : ix), cn = dpp<0x111>(hi, lp ? hi : in);  // row_shr:1
    const T dx = dpp<0x111>(lo, lp ? lo : jx), dn = dpp<0x111>(hi, lp ? hi : jn);
    const T ex = dpp<0x101>(lo, ls ? lo : kx), en = dpp<0x101>(hi, ls ? hi : kn);  // row_shl:1
#pragma unroll
    for (int i = 0; i < V; ++i) {
      px[i] = hmax(px[i], cx);
      pn[i] = hmin(pn[i], cn);
      qx[i] = hmax(qx[i], dx);
      qn[i] = hmin(qn[i], dn);
      sx[i] = hmax(sx[i], ex);
      sn[i] = hmin(sn[i], en);
    }
  }
#pragma unroll
  for (int i = 0; i < V; ++i) {
    if constexpr (WX) {
      hpx[lds_idx<T>(lane * V + i)] = px[i];
      hpx[lds_idx<T>(W + lane * V + i)] = qx[i];
    }
    if constexpr (WN) {
      hpn[lds_idx<T>(lane * V + i)] = pn[i];
      hpn[lds_idx<T>(W + lane * V + i)] = qn[i];
    }
  }
  f2_wave_sync();
#pragma unroll
  for (int i = 0; i < V; ++i) {
    const int cc = lane * V + i, e = cc + wc - 1, b1 = cc >> lgBh;
    if constexpr (WX) rx[i] = hmax(sx[i], hpx[lds_idx<T>(e)]);
    if constexpr (WN) rn[i] = hmin(sn[i], hpn[lds_idx<T>(e)]);
    // whole blocks b1+1 .. inside the window; past the last one the
    // index clamps to e, whose PRE is already taken
#pragma unroll
    for (int k = 1; k <= (KM > 0 ? KM : kmax); ++k) {
      const int mi = min((((b1 + k + 1) << lgBh) - 1), e);
      if constexpr (WX) rx[i] = hmax(rx[i], hpx[lds_idx<T>(mi)]);
      if constexpr (WN) rn[i] = hmin(rn[i], hpn[lds_idx<T>(mi)]);
    }
  }
}

// COLS: column-only mode, the input being the pair of row-filtered images
// (the second pass of rows-then-columns): the same column filter, no row
// work, no halo columns.  OUT: 3 both outputs, 1 max only, 2 min only (the
// other side's LDS, loads and arithmetic are compiled out).
template <class T, int B, int V, int KM, bool VIN, bool COLS, int OUT>
__global__ __launch_bounds__(64) void k_f2d(F2dArgs<typename F2Store<T>::S> a) {
  constexpr bool WX = (OUT & 1) != 0, WN = (OUT & 2) != 0;
  constexpr int W = 64 * V;                     // lane positions per strip (x2 columns when packed)
  constexpr int RB = 2 * B;                     // ring rows
  // input rows in flight (packed 16-bit rows are half as many bytes per
  // lane; MI355X, 8192^2: two rows ahead beat four for them at V = 4)
  constexpr int D = V >= 8 ? 2 : (V >= 4 ? (F2Store<T>::halves == 2 ? 2 : 4) : 8);
  __shared__ T ringx[WX ? RB * W : 1], ringn[WN ? RB * W : 1];  // [slot][i][lane]
  __shared__ T hpx[WX ? lds_len<T>(2 * W) : 1], hpn[WN ? lds_len<T>(2 * W) : 1];  // row PRE, strip + halo
  const int lane = threadIdx.x;
  // consecutive tiles on one XCD (workgroups are dealt round robin over
  // the 8 XCDs), so neighbouring strips share their halo columns in L2
  const int64_t per = gridDim.x / 8;
  const int64_t tile = (int64_t)(blockIdx.x & 7) * per + (blockIdx.x >> 3);
  if (tile >= a.ntiles) return;
  const int64_t band = tile / a.strips, strip = tile - band * a.strips;
  const int64_t orows = a.rows - a.wr + 1, oc = a.cols - a.wc + 1;
  const int64_t c0 = strip * W * F2Store<T>::halves, r0 = band * (int64_t)a.TR;
  const int nr = (int)min((int64_t)a.TR, orows - r0);  // output rows of the band
  const int NR = nr + a.wr - 1;                        // input rows streamed
  const int wr = a.wr, wc = a.wc;
  // along the row: blocks of Bh <= 16 V columns, so a block's lanes lie in
  // one 16-lane DPP row (no cross-row steps); a window then covers up to
  // KM whole blocks, whose aggregates are PRE at their last columns
  const int lgBh = 31 - __builtin_clz((unsigned)min(wc, 16 * V));
  const int Bh = 1 << lgBh;
  const int mh = Bh > V ? Bh / V : 1;  // lanes per block, <= 16
  const int lig = lane & (mh - 1);
  const int kmax = max(0, (wc + Bh - 2) / Bh - 1);
  // the column suffix of the window's first row read before the row work
  // (both outputs; with one output the registers it holds cost more)
  constexpr bool EARLY = OUT == 3;
  // down the columns: blocks of B rows (wr <= 2B)
  constexpr int lgB = B == 1 ? 0 : (B == 2 ? 1 : (B == 4 ? 2 : (B == 8 ? 3 : (B == 16 ? 4 : 5))));

  F2Raw<T, V> buf[D];
#pragma unroll
  for (int d = 0; d < D; ++d)
    if (d < NR) {
      if constexpr (COLS) f2_pair_issue<T, V, VIN, OUT>(a, r0 + d, c0, buf[d]);
      else f2_row_issue<T, V, VIN>(a, r0 + d, c0, buf[d]);
    }
  T Px[V], Pn[V], Ax[V], An[V];  // running column PRE; aggregate of the last whole block
#pragma unroll
  for (int i = 0; i < V; ++i) {
    Px[i] = Ax[i] = Lim<T>::lo();
    Pn[i] = An[i] = Lim<T>::hi();
  }
  for (int t0 = 0; t0 < NR; t0 += D) {
#pragma unroll
    for (int d = 0; d < D; ++d) {
      const int t = t0 + d;
      if (t < NR) {
        // ---- down the columns, first part: the block before this row is
        // complete at a block start: its suffixes, in place
        const int slot = t & (RB - 1);
        const bool bstart = (t & (B - 1)) == 0;
        if (bstart && t > 0) {
          const int s0 = (t - B) & (RB - 1);
#pragma unroll
          for (int i = 0; i < V; ++i) {
            if constexpr (WX) {
              T ux = ringx[((s0 + B - 1) * V + i) * 64 + lane];
              for (int k = B - 2; k >= 0; --k) {
                const int ix = ((s0 + k) * V + i) * 64 + lane;
                ux = hmax(ux, ringx[ix]);
                ringx[ix] = ux;
              }
              Ax[i] = ux;
            }
            if constexpr (WN) {
              T un = ringn[((s0 + B - 1) * V + i) * 64 + lane];
              for (int k = B - 2; k >= 0; --k) {
                const int ix = ((s0 + k) * V + i) * 64 + lane;
                un = hmin(un, ringn[ix]);
                ringn[ix] = un;
              }
              An[i] = un;
            }
          }
        }
        // the suffix at the first row j of the window ending here, read
        // before the row work so that its latency overlaps it (read in every
        // row, used where the window starts in an earlier block)
        const int j = t - wr + 1, bj = j >> lgB, bt = t >> lgB;
        const int js = j & (RB - 1);
        T sjx[V], sjn[V];
        if constexpr (EARLY) {
#pragma unroll
          for (int i = 0; i < V; ++i) {
            sjx[i] = ringx[(js * V + i) * 64 + lane];
            sjn[i] = ringn[(js * V + i) * 64 + lane];
          }
        }
        T rx[V], rn[V];  // the row-filtered values of this lane's columns
        if constexpr (COLS) {
          f2_pair_take<T, V, OUT>(buf[d], rx, rn);
          if (t + D < NR) f2_pair_issue<T, V, VIN, OUT>(a, r0 + t + D, c0, buf[d]);
        } else {
          // ---- along the row
          T x[V], h[V];
          f2_row_take<T, V>(buf[d], x, h);
          f2_row_filter<T, V, KM, WX, WN>(x, h, wc, lgBh, mh, lig, kmax, hpx, hpn, rx, rn);
          f2_wave_sync();  // the row buffer is rewritten by the next row
          // the next loads into this slot of the row queue
          if (t + D < NR) f2_row_issue<T, V, VIN>(a, r0 + t + D, c0, buf[d]);
        }
        // ---- down the columns: this row into the ring and the running PRE
#pragma unroll
        for (int i = 0; i < V; ++i) {
          if constexpr (WX) ringx[(slot * V + i) * 64 + lane] = rx[i];
          if constexpr (WN) ringn[(slot * V + i) * 64 + lane] = rn[i];
          const T ax = hmax(Px[i], rx[i]), an = hmin(Pn[i], rn[i]);
          Px[i] = bstart ? rx[i] : ax;
          Pn[i] = bstart ? rn[i] : an;
        }
        if (t >= wr - 1) {
          // the window of rows [j, t] is complete
          const bool use_s = bt > bj, use_a = bt > bj + 1;
          T ox[V], on[V];
#pragma unroll
          for (int i = 0; i < V; ++i) {
            if constexpr (!EARLY) {
              if (use_s) {
                if constexpr (WX) sjx[i] = ringx[(js * V + i) * 64 + lane];
                if constexpr (WN) sjn[i] = ringn[(js * V + i) * 64 + lane];
              } else {
                sjx[i] = Px[i];
                sjn[i] = Pn[i];
              }
            }
            const T mx = hmax(Px[i], sjx[i]), mn = hmin(Pn[i], sjn[i]);
            ox[i] = use_s ? mx : Px[i];
            on[i] = use_s ? mn : Pn[i];
            const T ax = hmax(ox[i], Ax[i]), an = hmin(on[i], An[i]);
            ox[i] = use_a ? ax : ox[i];
            on[i] = use_a ? an : on[i];
          }
          const int64_t cm = c0 + lane * V, orow = r0 + j;
          if constexpr (WX) f2_out_store<T, V>(a.omax + orow * a.ld_out, cm, oc, ox);
          if constexpr (WN) f2_out_store<T, V>(a.omin + orow * a.ld_out, cm, oc, on);
        }
      }
    }
  }
}

// Column blocks B (largest power of two <= w_rows, at most 32) and lane
// widths V: the ring is 2B x 64V elements per image per wavefront, so V
// trades the per-column cost of the row scans against LDS occupancy.  On
// MI355X (8192^2 float32 / uint16, w = 3 and 15) V = 4 (B <= 4), 2 (B = 8)
// and 1 beat twice those widths by 10-40% and half of them by up to 30%.
inline int f2d_V(int B, size_t) { return B >= 16 ? 1 : (B >= 8 ? 2 : 4); }
inline size_t f2d_size(int dtype) { return dtype == 1 ? 8 : (dtype == 3 ? 2 : 4); }


// Row starts aligned to the access width (min(16, V * s) bytes): the
// kernels' vector loads.
template <class T, int V> bool f2_vin(const F2dArgs<typename F2Store<T>::S>& a) {
  using S = typename F2Store<T>::S;
  const size_t al = std::min<size_t>(16, (size_t)V * sizeof(S));
  return al >= 4 && (uintptr_t)a.in % al == 0 && (uintptr_t)a.in2 % al == 0 &&
         ((size_t)a.ld_in * sizeof(S)) % al == 0;
}

template <class T, int B, int V, bool COLS, int OUT>
hipError_t f2d_go(const F2dArgs<typename F2Store<T>::S>& a, int64_t grid, hipStream_t st) {
  const bool vin = f2_vin<T, V>(a);
  auto go = [&](auto km) {
    constexpr int KM = decltype(km)::value;
    if (vin) hipLaunchKernelGGL((k_f2d<T, B, V, KM, true, COLS, OUT>), dim3((unsigned)grid), dim3(64), 0, st, a);
    else hipLaunchKernelGGL((k_f2d<T, B, V, KM, false, COLS, OUT>), dim3((unsigned)grid), dim3(64), 0, st, a);
    return hipGetLastError();
  };
  if constexpr (COLS) {
    return go(std::integral_constant<int, 1>());  // no row work
  } else if constexpr (OUT != 3) {
    return go(std::integral_constant<int, 0>());  // one output: the loop over whole row blocks
  } else {
    // both outputs: a fixed count of whole row blocks, up to four when a
    // window is wider than 16 V columns
    if (a.wc > 16 * V) return go(std::integral_constant<int, 4>());
    return go(std::integral_constant<int, 1>());
  }
}

// Shared launcher: COLS = column-only mode (in, in2: the row-filtered max
// and min images, w_cols = 1); OUT as in k_f2d.  Instantiated in one
// translation unit per OUT (compiled in parallel).
template <bool COLS, int OUT>
hipError_t f2d_launch(int dtype, const void* d_in, const void* d_in2, int64_t ld_in, int64_t rows,
                             int64_t cols, int64_t w_rows, int64_t w_cols, void* d_max, void* d_min, int64_t ld_out,
                             int64_t band_rows, hipStream_t st) {
  const int64_t orows = rows - w_rows + 1, oc = cols - w_cols + 1;
  if (orows <= 0 || oc <= 0) return hipSuccess;
  int B = 1;
  while (2 * B <= w_rows) B *= 2;
  const int V = f2d_V(B, f2d_size(dtype));
  const int W = 64 * V * (dtype == 3 ? 2 : 1);  // output columns per strip (16-bit data: two halves)
  const int64_t strips = (oc + W - 1) / W;
  // bands: about four waves per SIMD over the chip when the image allows,
  // at least 4B rows each so the w_rows-1 halo rows stay a small share;
  // for w_rows < 4 at most 16 rows and for 16-bit data with 8 <= w_rows <
  // 16 and both outputs at most 32 (MI355X, 8192^2: w = 3 float32 0.215 ->
  // 0.186 ms, uint16 0.139 -> 0.124 against the rule's 64- and 32-row
  // bands; uint16 w = 11 / 15 0.24 -> 0.21 / 0.22 against 64 rows, while
  // one output keeps 64: 0.121 against 0.136 ms at w = 15; elsewhere the
  // rule's bands were within 2% of the best, one output or two)
  int64_t TR = band_rows;
  if (TR <= 0) {
    const int64_t target = 4 * 4 * 256;
    const int64_t bands = std::max<int64_t>(1, target / strips);
    TR = std::max<int64_t>((orows + bands - 1) / bands, 4 * B);
    if (B <= 2) TR = std::min<int64_t>(TR, 16);
    if (dtype == 3 && B == 8 && OUT == 3) TR = std::min<int64_t>(TR, 32);
  }
  TR = std::min<int64_t>(TR, orows);
  if (TR > (1 << 30)) return hipErrorNotSupported;
  const int64_t bands = (orows + TR - 1) / TR;
  const int64_t ntiles = strips * bands;
  const int64_t grid = (ntiles + 7) / 8 * 8;
  if (grid > 0x7fffffff) return hipErrorNotSupported;
  auto go = [&](auto* p) -> hipError_t {
    using T = std::remove_pointer_t<decltype(p)>;  // lane value type
    using S = typename F2Store<T>::S;              // image element type
    F2dArgs<S> a;
    a.in = (const S*)d_in;
    a.in2 = (const S*)d_in2;
    a.ld_in = ld_in;
    a.rows = rows;
    a.cols = cols;
    a.wr = (int)w_rows;
    a.wc = (int)w_cols;
    a.omax = (S*)d_max;
    a.omin = (S*)d_min;
    a.ld_out = ld_out;
    a.strips = (int)strips;
    a.TR = (int)TR;
    a.ntiles = ntiles;
    switch (B) {
      case 1: return f2d_go<T, 1, 4, COLS, OUT>(a, grid, st);
      case 2: return f2d_go<T, 2, 4, COLS, OUT>(a, grid, st);
      case 4: return f2d_go<T, 4, 4, COLS, OUT>(a, grid, st);
      case 8: return f2d_go<T, 8, 2, COLS, OUT>(a, grid, st);
      case 16: return f2d_go<T, 16, 1, COLS, OUT>(a, grid, st);
      default: return f2d_go<T, 32, 1, COLS, OUT>(a, grid, st);
    }
  };
  switch (dtype) {
    case 0: return go((float*)nullptr);
    case 1: return go((double*)nullptr);
    case 2: return go((int32_t*)nullptr);
    case 3: return go((P16*)nullptr);
    default: return hipErrorInvalidValue;
  }
}


// one translation unit each
extern template hipError_t f2d_launch<false, 1>(int, const void*, const void*, int64_t, int64_t, int64_t, int64_t,
                                                int64_t, void*, void*, int64_t, int64_t, hipStream_t);
extern template hipError_t f2d_launch<true, 1>(int, const void*, const void*, int64_t, int64_t, int64_t, int64_t,
                                               int64_t, void*, void*, int64_t, int64_t, hipStream_t);
extern template hipError_t f2d_launch<false, 2>(int, const void*, const void*, int64_t, int64_t, int64_t, int64_t,
                                                int64_t, void*, void*, int64_t, int64_t, hipStream_t);
extern template hipError_t f2d_launch<true, 2>(int, const void*, const void*, int64_t, int64_t, int64_t, int64_t,
                                               int64_t, void*, void*, int64_t, int64_t, hipStream_t);
extern template hipError_t f2d_launch<false, 3>(int, const void*, const void*, int64_t, int64_t, int64_t, int64_t,
                                                int64_t, void*, void*, int64_t, int64_t, hipStream_t);
extern template hipError_t f2d_launch<true, 3>(int, const void*, const void*, int64_t, int64_t, int64_t, int64_t,
                                               int64_t, void*, void*, int64_t, int64_t, hipStream_t);

}  // namespace mm
