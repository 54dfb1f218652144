// gfx950 kernels of the 1-D running max-min filter.
//
// Both strategies rest on the block decomposition of van Herk and
// Gil-Werman (Related Work; Table 1): cut the series into blocks of B
// consecutive elements; for a window [j, j+w) that starts in block b1 and
// ends in block b2,
//     max a[j..j+w) = max( SUF[j], AGG[b1+1 .. b2-1], PRE[j+w-1] )
// where SUF[j] is the maximum from j to the end of its block, PRE[e] the
// maximum from the start of e's block to e, and AGG[b] a whole block's
// maximum (likewise for the minimum).  With B = w this is the classical
// form (no middle term).  All of it is selection: results are exact.
//
// * Tile strategy (k_tile, w <= 8192).  A persistent workgroup of 256
//   threads streams through a run of consecutive sub-tiles of 2048 windows,
//   each thread holding 8 consecutive positions in registers (16-byte loads,
//   the next sub-tile's loads in flight while the current one is scanned).
//   For w <= 2048, B is the largest power of two <= min(w, 1024), so w <= 2B
//   and at most one whole block lies inside a window; in-thread scans plus
//   DPP lane-group scans give PRE/SUF (B = 1024 folds two wavefronts through
//   LDS).  PRE goes to an LDS ring of two sub-tiles, SUF stays in registers,
//   and the windows starting in the previous sub-tile are stored with
//   shifted 16-byte stores.  LAG = 2..4 (w <= 4096 / 6144 / 8192) take whole
//   sub-tiles as blocks and keep the SUF of LAG sub-tiles in registers.
//   Job kinds: one series (optionally two segments: a stream's carry plus
//   its chunk), described series of a batch, rows of a 2-D image.
//
// * Chunk strategy (k_chunk, batched windows past the tile kernel, forced
//   for tests).  Blocks of exactly w inputs aligned at the series start, cut
//   into K chunks of C <= 4096.  The workgroup that owns input chunk (b, k)
//   emits every window that ENDS in it (the zero-latency view of Section 1
//   applied to chunks): PRE from its own chunk plus the aggregates of chunks
//   (b, 0..k-1), SUF from re-reading chunk (b-1, k) plus the aggregates of
//   chunks (b-1, k+1..K-1).  Chunks are taken by in-order tickets; each
//   publishes its aggregate before waiting, and waits only on the K-1
//   chunks ticketed just before it, so every wait ends.
//
// * Long windows of one series (w > 8192).  k_chunk_col1: one pass, a
//   column of chunks per workgroup (K sibling columns run together under a
//   cooperative launch and exchange chunk records); k_chunk_agg +
//   k_chunk_col: the two-pass form (aggregates, then columns) for devices
//   where the cooperative grid does not fit; k_chunk with look-back on
//   request.
#include <type_traits>

#include "mm_launch.hpp"

namespace mm {

// ------------------------------------------------------------------ helpers
// XCD-aware static schedule: consecutive workgroup ids land on different
// XCDs (round robin over 8), so give XCD x the x-th eighth of the tiles, in
// order.  Neighbouring tiles then share an L2 (tile halos hit in cache).
__device__ __forceinline__ void xcd_schedule(int64_t ntiles, int64_t& first, int64_t& stride,
                                             int64_t& end) {
  const int NX = 8;
  const int g = blockIdx.x, G = gridDim.x;
  if (G < NX || ntiles < NX) {
    first = g;
    stride = G;
    end = ntiles;
    return;
  }
  const int x = g % NX, r = g / NX;
  const int gx = (G - x + NX - 1) / NX;
  first = ntiles * x / NX + r;
  stride = gx;
  end = ntiles * (x + 1) / NX;
}

// Last k in [0, S-1] with pre[k] <= t, given pre[0] <= t < pre[S]; pre is
// non-decreasing.  Every wavefront searches independently (64-ary).
__device__ int64_t find_series(const int64_t* pre, int64_t S, int64_t t) {
  const int lane = threadIdx.x & 63;
  int64_t lo = 0, hi = S - 1;
  while (hi > lo) {
    const int64_t span = hi - lo;
    const int64_t step = span < 64 ? 1 : (span + 63) / 64;
    int64_t idx = lo + (int64_t)lane * step;
    if (idx > hi) idx = hi;
    const bool p = pre[idx] <= t;
    const uint64_t m = __ballot(p);
    const int L = 63 - __builtin_clzll(m);
    int64_t nlo = lo + (int64_t)L * step;
    if (nlo > hi) nlo = hi;
    int64_t nhi = hi;
    if (L < 63) {
      const int64_t c = lo + (int64_t)(L + 1) * step - 1;
      if (c < nhi) nhi = c;
    }
    lo = nlo;
    hi = nhi;
  }
  return lo;
}

// What one launch works on: a single series, S described series (packed
// buffer with descriptors and per-strategy tile prefix sums), or `rows`
// equal-length series at a fixed stride (the row pass of the 2-D filter).
enum JobMode : int { kJobOne = 0, kJobDescs = 1, kJobRows = 2 };

template <int MODE, class T>
__device__ __forceinline__ int64_t job_tiles(const Job<T>& j) {
  return MODE == kJobDescs ? j.pre[j.S] : j.ntiles;
}

// Series of global tile t, its tile index inside the series, and the global
// index of the series' first tile.
template <int MODE, class T>
__device__ __forceinline__ Series<T> job_series(const Job<T>& j, int64_t t, int64_t& local, int64_t& gbase) {
  if constexpr (MODE == kJobOne) {
    local = t;
    gbase = 0;
    return j.one;
  } else if constexpr (MODE == kJobDescs) {
    const int64_t k = find_series(j.pre, j.S, t);
    gbase = j.pre[k];
    local = t - gbase;
    return j.descs[k];
  } else {
    const int64_t k = t / j.tpr;
    gbase = k * j.tpr;
    local = t - gbase;
    Series<T> s;
    s.a = j.in + k * j.ld_in;
    s.b = s.a;  // never read (na = n); not null, which the optimiser would treat as unreachable
    s.na = j.n;
    s.n = j.n;
    s.w = j.w;
    s.omax = j.omax ? j.omax + k * j.ld_out : nullptr;  // a null output is not computed
    s.omin = j.omin ? j.omin + k * j.ld_out : nullptr;
    s.carry = nullptr;
    return s;
  }
}

// ============================================================ tile strategy
// A workgroup streams through a run of consecutive windows [R0, R1), one
// sub-tile of kTileOut positions at a time.  Every thread owns 8 consecutive
// positions of the sub-tile and loads them straight into registers (16-byte
// loads when aligned; the next sub-tile's loads are issued before the
// current one is computed).  For sub-tile P_k it computes
//   PRE over P_k (written to an LDS ring of two sub-tiles), and
//   SUF over P_k (kept in registers until the next sub-tile),
// then emits the windows that START in P_{k-1}: their ends lie in P_{k-1} or
// P_k (w - 1 <= kTileOut), whose PRE values are both in the ring.  Each input
// is read from memory once; only a run's last sub-tile overlaps the next run.
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

template <class T, bool COMPACT = false> struct TileLds {
  T pm[lds_len<T>(2 * kTileOut)];  // PRE (max) ring, indexed by position mod 2*kTileOut
  T pn[lds_len<T>(2 * kTileOut)];  // PRE (min) ring
  T wt[4][kTileThreads / 64];      // wavefront totals (blocks of two or four wavefronts)
  T st[2][8];                      // LAG >= 3: sub-tile totals, indexed by sub-tile mod 8
};
// With locations at LAG 1: a PRE entry's location lies at most 2047
// positions before its own (inside its block), so the rings keep the value
// and that distance as 16 bits, 6 bytes an entry for 4-byte data instead of
// 8 (f32: 50.7 instead of 66.6 KiB, three workgroups per CU instead of two;
// MI355X, n = 2^28: w = 1024 2.12 -> 1.94 ms, 2048 2.26 -> 1.99; at LAG 2,
// held to two workgroups by its registers, it was 2% slower).
template <class T> struct TileLds<Loc<T>, true> {
  T pmv[lds_len<T>(2 * kTileOut)];
  T pnv[lds_len<T>(2 * kTileOut)];
  uint16_t pmd[lds_len<uint16_t>(2 * kTileOut)];
  uint16_t pnd[lds_len<uint16_t>(2 * kTileOut)];
  Loc<T> wt[4][kTileThreads / 64];
  Loc<T> st[2][8];
};
// ring access: slot (ring index) of position pos (relative to the run start)
template <class T> __device__ __forceinline__ void ring_put(TileLds<T, false>& sm, int slot, int, T x, T n) {
  sm.pm[lds_idx<T>(slot)] = x;
  sm.pn[lds_idx<T>(slot)] = n;
}
template <class T>
__device__ __forceinline__ void ring_put(TileLds<Loc<T>, true>& sm, int slot, int pos, Loc<T> x, Loc<T> n) {
  sm.pmv[lds_idx<T>(slot)] = x.v;
  sm.pnv[lds_idx<T>(slot)] = n.v;
  sm.pmd[lds_idx<uint16_t>(slot)] = (uint16_t)(pos - x.i);
  sm.pnd[lds_idx<uint16_t>(slot)] = (uint16_t)(pos - n.i);
}
template <class T> __device__ __forceinline__ T ring_x(const TileLds<T, false>& sm, int slot, int) {
  return sm.pm[lds_idx<T>(slot)];
}
template <class T> __device__ __forceinline__ T ring_n(const TileLds<T, false>& sm, int slot, int) {
  return sm.pn[lds_idx<T>(slot)];
}
template <class T> __device__ __forceinline__ Loc<T> ring_x(const TileLds<Loc<T>, true>& sm, int slot, int pos) {
  return Loc<T>{sm.pmv[lds_idx<T>(slot)], pos - (int)sm.pmd[lds_idx<uint16_t>(slot)]};
}
template <class T> __device__ __forceinline__ Loc<T> ring_n(const TileLds<Loc<T>, true>& sm, int slot, int pos) {
  return Loc<T>{sm.pnv[lds_idx<T>(slot)], pos - (int)sm.pnd[lds_idx<uint16_t>(slot)]};
}

// Series and outputs need not be 16-byte aligned (a packed batch puts
// series at arbitrary element offsets).  A wavefront covers 64 * 8
// consecutive positions, a multiple of 16 bytes, so all its lanes share one
// misalignment D (in elements): lanes then load (store) the aligned 16-byte
// vectors shifted by D and pass the D elements that cross a lane boundary to
// the neighbouring lane with one shuffle each; the wavefront's edge lanes
// load (store) those few elements singly.

// An empty statement that reads x: the compiler waits for x's load right
// here (and knows it needs no later wait), instead of where x is next read.
template <class T> __device__ __forceinline__ void settle(const T& x) {
  if constexpr (sizeof(T) == 8) {
    uint64_t u;
    __builtin_memcpy(&u, &x, 8);
    asm volatile("" ::"v"(u));
  } else {
    uint32_t u = 0;
    __builtin_memcpy(&u, &x, sizeof(T));
    asm volatile("" ::"v"(u));
  }
}

// Workgroup barrier ordering LDS only.  The tile kernel's wavefronts share
// nothing through global memory; __syncthreads would also make each
// wavefront wait for its outstanding global stores to complete.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Elements a lane may need beyond its aligned vectors (the largest shift).
template <class T> constexpr int kTileEx = 16 / (int)sizeof(T) - 1;

// Issue the loads of the 8 inputs at positions p .. p+7 and nothing else,
// so the sub-tile's prefetch stays in flight while the current one is
// computed.  Where the wavefront's positions lie in the segment vb below
// lim, v gets the aligned 16-byte vectors holding p - d .. p - d + 7 (the
// same instructions whatever the misalignment d, so no branch joins two
// sets of loaded registers) and lane 63 the d inputs after them in ex; the
// result is true when run_fix must still shift them by d.  Elsewhere
// (a run's end, a series split over two buffers) v gets the inputs one by
// one, those >= lim as 0 (never used).
template <class T>
__device__ __forceinline__ bool run_issue(const Series<T>& s, const T* vb, int d, int64_t p, int64_t lim,
                                          T (&v)[kTileV], T (&ex)[kTileEx<T>]) {
  constexpr int V = kTileV, EV = 16 / (int)sizeof(T);
  const int64_t pw = p - (int64_t)(threadIdx.x & 63) * V;  // the wavefront's first position
  // the same for every lane; readfirstlane lets the compiler see that, so
  // the branches here and on the result are plain jumps, not two masked
  // halves it has to assume may both be skipped
  const bool vec = __builtin_amdgcn_readfirstlane((int)(vb != nullptr && pw + 64 * V <= lim)) != 0;
  if (vec) {
#pragma unroll
    for (int k = 0; k < V / EV; ++k) {
      const u32x4 u = gload((const u32x4*)(vb + p - d + k * EV));
      __builtin_memcpy(&v[k * EV], &u, 16);
    }
    if ((threadIdx.x & 63) == 63) {
#pragma unroll
      for (int j = 0; j < kTileEx<T>; ++j)
        if (j < d) ex[j] = gload(vb + p + V - d + j);
    }
    return d != 0;
  }
#pragma unroll
  for (int i = 0; i < V; ++i) v[i] = (p + i < lim) ? src_at(s, p + i) : T(0);
  return false;
}

// v[i] = input p + i from the vectors run_issue loaded at p - D: the D
// inputs that cross into the next lane come from it by one shuffle each
// (lane 63: from ex).
template <class T, int D>
__device__ __forceinline__ void shift_in(T (&v)[kTileV], const T (&ex)[kTileEx<T>]) {
  constexpr int V = kTileV;
  T nb[D];
#pragma unroll
  for (int j = 0; j < D; ++j) nb[j] = shdn(v[j], 1, 64);
#pragma unroll
  for (int i = 0; i < V - D; ++i) v[i] = v[i + D];
  const bool last = (threadIdx.x & 63) == 63;
#pragma unroll
  for (int i = V - D; i < V; ++i) v[i] = last ? ex[i - (V - D)] : nb[i - (V - D)];
}

template <class T>
__device__ __forceinline__ void run_fix(int d, T (&v)[kTileV], const T (&ex)[kTileEx<T>]) {
  constexpr int EV = 16 / (int)sizeof(T);
  switch (d) {
    case 1: shift_in<T, 1>(v, ex); break;
    case 2: if constexpr (EV > 2) shift_in<T, 2>(v, ex); break;
    case 3: if constexpr (EV > 3) shift_in<T, 3>(v, ex); break;
    case 4: if constexpr (EV > 4) shift_in<T, 4>(v, ex); break;
    case 5: if constexpr (EV > 5) shift_in<T, 5>(v, ex); break;
    case 6: if constexpr (EV > 6) shift_in<T, 6>(v, ex); break;
    case 7: if constexpr (EV > 7) shift_in<T, 7>(v, ex); break;
    default: break;
  }
}

// store o[i] at out[i] (i < 8) with aligned vectors starting at out + D
template <class T, int D>
__device__ __forceinline__ void store_shifted(T* out, const T (&o)[kTileV]) {
  constexpr int V = kTileV, EV = 16 / (int)sizeof(T);
  const int lane = threadIdx.x & 63;
  T nb[D];
#pragma unroll
  for (int j = 0; j < D; ++j) nb[j] = shdn(o[j], 1, 64);
#pragma unroll
  for (int k = 0; k < V / EV; ++k) {
    if (D + (k + 1) * EV > V && lane == 63) {
      // the vector would reach into the next wavefront's positions
#pragma unroll
      for (int i = D + k * EV; i < V; ++i) gstore(out + i, o[i]);
    } else {
      T e[EV];
#pragma unroll
      for (int x = 0; x < EV; ++x) {
        const int i = D + k * EV + x;
        e[x] = i < V ? o[i] : nb[i - V];
      }
      u32x4 u;
      __builtin_memcpy(&u, e, 16);
      gstore((u32x4*)(out + D + k * EV), u);
    }
  }
  if (lane == 0) {
#pragma unroll
    for (int i = 0; i < D; ++i) gstore(out + i, o[i]);
  }
}

// Store the 8 outputs of positions q .. q+7 (only those < R1).  om or on
// may be null (that output is not wanted).  ovec: the outputs present share
// the misalignment d (elements) at position q.
template <class T>
__device__ __forceinline__ void run_store(T* om, T* on, bool ovec, int d, int64_t q, int64_t R1,
                                          const T (&ox)[kTileV], const T (&on_)[kTileV]) {
  constexpr int V = kTileV, EV = 16 / (int)sizeof(T);
  const int64_t qw = q - (int64_t)(threadIdx.x & 63) * V;
  if (ovec && qw + 64 * V <= R1) {
    const int sh = (EV - d) & (EV - 1);  // elements before the first aligned vector
    switch (sh) {
      case 0:
#pragma unroll
        for (int k = 0; k < V / EV; ++k) {
          u32x4 a, b;
          __builtin_memcpy(&a, &ox[k * EV], 16);
          __builtin_memcpy(&b, &on_[k * EV], 16);
          if (om) gstore((u32x4*)(om + k * EV), a);
          if (on) gstore((u32x4*)(on + k * EV), b);
        }
        break;
#define MM_STORE_CASE(D)                        \
  case D:                                       \
    if constexpr (EV > D) {                     \
      if (om) store_shifted<T, D>(om, ox);      \
      if (on) store_shifted<T, D>(on, on_);     \
    }                                           \
    break;
      MM_STORE_CASE(1)
      MM_STORE_CASE(2)
      MM_STORE_CASE(3)
      MM_STORE_CASE(4)
      MM_STORE_CASE(5)
      MM_STORE_CASE(6)
      MM_STORE_CASE(7)
#undef MM_STORE_CASE
    }
  } else {
#pragma unroll
    for (int i = 0; i < V; ++i)
      if (q + i < R1) {
        if (om) gstore(om + i, ox[i]);
        if (on) gstore(on + i, on_[i]);
      }
  }
}

// ARG: also the leftmost location of every window's max and min (values
// travel with their location relative to R0; outputs amax/amin get R0 +
// location, the position in the series).
// LAG: sub-tiles between a window's first and last element.  LAG 1 (w <=
// 2048): blocks up to 1024, the windows starting in P_{k-1} are emitted
// once P_k is scanned.  LAG L >= 2 ((L-1) 2048 < w <= L 2048): blocks of
// one whole sub-tile (four wavefronts), the windows starting in P_{k-L} are
// emitted once P_k is scanned, so L sub-tiles of SUF stay in registers;
// their ends lie in P_{k-1} or P_k (PRE from the ring) and the whole
// sub-tiles between are one block (L = 2: PRE at its end, from the ring)
// or several (L >= 3: the totals of the last 8 sub-tiles, kept in LDS).
template <class T, bool ARG, int LAG>
__device__ __forceinline__ void run_body(const Series<T>& s, int64_t R0, int64_t R1,
                                         TileLds<typename ElemOf<T, ARG>::type, ARG && LAG == 1>& sm,
                                         int64_t* amax,
                                         int64_t* amin) {
  typedef typename ElemOf<T, ARG>::type E;
  E* const et = nullptr;  // selects elem()'s overload
  constexpr int NT = kTileThreads, V = kTileV, TT = kTileOut, RING = 2 * kTileOut;
  const int tid = threadIdx.x;
  const int w = (int)s.w;
  static_assert(LAG >= 1 && LAG <= 4, "emission lag of one to four sub-tiles");
  const int lgB = 31 - __builtin_clz((unsigned)min(w, LAG == 1 ? kTileMaxBlock : TT));
  const int B = 1 << lgB;
  const int m = B > V ? B / V : 1;  // lanes per block (128, 256: two, four wavefronts)
  const int mw = m < 64 ? m : 64;     // lanes per block within one wavefront
  const int lig = tid & (mw - 1);
  const int64_t nout = s.n - s.w + 1;
  const int64_t lim = min(s.n, R1 + (int64_t)w - 1);  // inputs used: [R0, lim)
  const int nsub = (int)((R1 - 1 - R0) / TT) + 1 + LAG;  // sub-tiles P_0 .. P_{nsub-1}
  // 16-byte loads when [R0, lim) lies in one source segment
  constexpr int EV = 16 / (int)sizeof(T);
  const T* vbase = nullptr;
  if (lim <= s.na) vbase = s.a;
  else if (R0 >= s.na) vbase = s.b - s.na;
  const int din = vbase != nullptr ? (int)(((uintptr_t)(vbase + R0) / sizeof(T)) & (EV - 1)) : 0;
  // either output may be null (max-only / min-only filter)
  const int dmx = s.omax ? (int)(((uintptr_t)(s.omax + R0) / sizeof(T)) & (EV - 1)) : -1;
  const int dmn = s.omin ? (int)(((uintptr_t)(s.omin + R0) / sizeof(T)) & (EV - 1)) : -1;
  const bool ovec = dmx < 0 || dmn < 0 || dmx == dmn;
  const int dout = dmx >= 0 ? dmx : dmn;
  const bool last_run = R1 == nout;

  T cur[V], nxt[V], ex[kTileEx<T>];
  E hx[LAG][V], hn[LAG][V];  // SUF of P_{k-1} (index 0) .. P_{k-LAG}
  // the first sub-tile is waited for before the loop, whose body cannot
  // tell these loads from its own prefetch and would wait for both
  const bool fix0 = run_issue<T>(s, vbase, din, R0 + tid * V, lim, cur, ex);
#pragma unroll
  for (int i = 0; i < V; ++i) settle(cur[i]);
#pragma unroll
  for (int j = 0; j < kTileEx<T>; ++j) settle(ex[j]);
  if (__builtin_amdgcn_readfirstlane((int)fix0) != 0) run_fix<T>(din, cur, ex);
  for (int k = 0; k < nsub; ++k) {
    const int pr0 = k * TT + tid * V;  // position of cur[0], relative to R0
    bool nfix = false;
    if (k + 1 < nsub) nfix = run_issue<T>(s, vbase, din, R0 + pr0 + TT, lim, nxt, ex);
    nfix = __builtin_amdgcn_readfirstlane((int)nfix) != 0;  // uniform: a jump, not masked halves
    if (s.carry != nullptr && last_run) {
      // the series' last w-1 inputs are the next push's carry
#pragma unroll
      for (int i = 0; i < V; ++i) {
        const int64_t p = R0 + pr0 + i;
        if (p >= nout && p < s.n) gstore(s.carry + (p - nout), cur[i]);
      }
    }
    // A sub-tile past the last input (a run's tail sub-tile) only emits the
    // windows of the one before; its own PRE and SUF are never read.
    const bool live = R0 + (int64_t)k * TT < lim;
    E ux[V], un[V];
    if (live) {
      // PRE of P_k: within the thread, then across the lanes of its block
      E px[V], pn[V];
      px[0] = elem(cur[0], pr0, et);
      pn[0] = px[0];
#pragma unroll
      for (int i = 1; i < V; ++i) {
        const bool start = ((pr0 + i) & (B - 1)) == 0;  // a block begins here
        const E c = elem(cur[i], pr0 + i, et);
        px[i] = start ? c : hmax(px[i - 1], c);
        pn[i] = start ? c : hmin(pn[i - 1], c);
      }
      if (m > 1) {
        // a block spans mw aligned lanes of the wavefront (all of it, and
        // then the next wavefront too, when m > 64): exclusive scan of the
        // lane totals
        E ix = px[V - 1], in = pn[V - 1];
        E cx, cn;
        if constexpr (!ARG) {
          seg_prefix2<T, true>(ix, in, mw, lig);
          cx = dpp<0x138>(Lim<T>::lo(), ix);  // wave_shr:1 (read only where lig > 0)
          cn = dpp<0x138>(Lim<T>::hi(), in);
        } else {
          for (int d = 1; d < mw; d <<= 1) {
            const E a = shup(ix, d, mw), b = shup(in, d, mw);
            if (lig >= d) {
              ix = hmax(ix, a);
              in = hmin(in, b);
            }
          }
          cx = shup(ix, 1, mw);
          cn = shup(in, 1, mw);
        }
        if (lig > 0) {
#pragma unroll
          for (int i = 0; i < V; ++i) {
            px[i] = hmax(px[i], cx);
            pn[i] = hmin(pn[i], cn);
          }
        }
      }
      // SUF of P_k, kept for the next sub-tile's outputs
      ux[V - 1] = elem(cur[V - 1], pr0 + V - 1, et);
      un[V - 1] = ux[V - 1];
#pragma unroll
      for (int i = V - 2; i >= 0; --i) {
        const bool end = ((pr0 + i + 1) & (B - 1)) == 0;  // a block ends here
        const E c = elem(cur[i], pr0 + i, et);
        ux[i] = end ? c : hmax(ux[i + 1], c);
        un[i] = end ? c : hmin(un[i + 1], c);
      }
      if (m > 1) {
        E jx = ux[0], jn = un[0];
        E cx, cn;
        if constexpr (!ARG) {
          seg_suffix2<T, true>(jx, jn, mw, lig);
          cx = dpp<0x130>(Lim<T>::lo(), jx);  // wave_shl:1 (read only where lig < mw-1)
          cn = dpp<0x130>(Lim<T>::hi(), jn);
        } else {
          for (int d = 1; d < mw; d <<= 1) {
            const E a = shdn(jx, d, mw), b = shdn(jn, d, mw);
            if (lig + d < mw) {
              jx = hmax(jx, a);
              jn = hmin(jn, b);
            }
          }
          cx = shdn(jx, 1, mw);
          cn = shdn(jn, 1, mw);
        }
        if (lig < mw - 1) {
#pragma unroll
          for (int i = 0; i < V; ++i) {
            ux[i] = hmax(ux[i], cx);
            un[i] = hmin(un[i], cn);
          }
        }
      }
      if (m > 64) {
        // blocks of G = m/64 wavefronts: each takes the totals of the
        // block's earlier wavefronts into its PRE and of its later ones
        // into its SUF (wavefront-uniform branches)
        const int lane = tid & 63, wv = tid >> 6, G = m >> 6, g0 = wv & ~(G - 1);
        if (lane == 63) {
          sm.wt[0][wv] = px[V - 1];
          sm.wt[1][wv] = pn[V - 1];
        }
        if (lane == 0) {
          sm.wt[2][wv] = ux[0];
          sm.wt[3][wv] = un[0];
        }
        __syncthreads();
        if (wv > g0) {
          E cx = sm.wt[0][g0], cn = sm.wt[1][g0];
          for (int o = g0 + 1; o < wv; ++o) {
            cx = hmax(cx, sm.wt[0][o]);
            cn = hmin(cn, sm.wt[1][o]);
          }
#pragma unroll
          for (int i = 0; i < V; ++i) {
            px[i] = hmax(px[i], cx);
            pn[i] = hmin(pn[i], cn);
          }
        }
        if (wv < g0 + G - 1) {
          E cx = sm.wt[2][g0 + G - 1], cn = sm.wt[3][g0 + G - 1];
          for (int o = g0 + G - 2; o > wv; --o) {
            cx = hmax(cx, sm.wt[2][o]);
            cn = hmin(cn, sm.wt[3][o]);
          }
#pragma unroll
          for (int i = 0; i < V; ++i) {
            ux[i] = hmax(ux[i], cx);
            un[i] = hmin(un[i], cn);
          }
        }
      }
      const int slot = pr0 & (RING - 1);
#pragma unroll
      for (int i = 0; i < V; ++i) {
        ring_put(sm, slot + i, pr0 + i, px[i], pn[i]);
      }
      if constexpr (LAG >= 3) {
        if (tid == NT - 1) {  // PRE at the sub-tile's last position: its total
          sm.st[0][k & 7] = px[V - 1];
          sm.st[1][k & 7] = pn[V - 1];
        }
      }
      __syncthreads();  // PRE of P_k visible
    }
    // The next sub-tile's inputs are waited for here, on every path (a wait
    // the compiler could see skipped would land after the stores, and one
    // counter covers loads and stores: it would wait for them too).
#pragma unroll
    for (int i = 0; i < V; ++i) settle(nxt[i]);
#pragma unroll
    for (int j = 0; j < kTileEx<T>; ++j) settle(ex[j]);
    if (nfix) run_fix<T>(din, nxt, ex);
    if (k >= LAG) {
      // windows starting in P_{k-LAG}: SUF (registers), PRE at the window
      // end and the whole block strictly inside, if any (both from the ring;
      // the ends lie in P_{k-1} or P_k)
      const int qr0 = pr0 - LAG * TT;
      // LAG >= 3: totals of the whole sub-tiles between P_{k-LAG} and the
      // window's last sub-tile, P_{k-1} (mx1) or P_k (mx0)
      E mx1 = elem(Lim<T>::lo(), 0, et), mn1 = elem(Lim<T>::hi(), 0, et), mx0 = mx1, mn0 = mn1;
      if constexpr (LAG >= 3) {
        for (int j = k - LAG + 1; j <= k - 2; ++j) {
          mx1 = hmax(mx1, sm.st[0][j & 7]);
          mn1 = hmin(mn1, sm.st[1][j & 7]);
        }
        mx0 = hmax(mx1, sm.st[0][(k - 1) & 7]);
        mn0 = hmin(mn1, sm.st[1][(k - 1) & 7]);
      }
      E ox[V], on[V];
#pragma unroll
      for (int i = 0; i < V; ++i) {
        const int q = qr0 + i, e = q + w - 1;
        E rx = hmax(hx[LAG - 1][i], ring_x(sm, e & (RING - 1), e));
        E rn = hmin(hn[LAG - 1][i], ring_n(sm, e & (RING - 1), e));
        const int b1 = q >> lgB, b2 = e >> lgB;
        if constexpr (LAG >= 3) {
          const bool last = b2 == b1 + LAG;  // ends in P_k
          rx = hmax(rx, last ? mx0 : mx1);
          rn = hmin(rn, last ? mn0 : mn1);
        } else if (b2 >= b1 + 2) {
          const int mp = ((b1 + 2) << lgB) - 1;  // the whole block's last position
          rx = hmax(rx, ring_x(sm, mp & (RING - 1), mp));
          rn = hmin(rn, ring_n(sm, mp & (RING - 1), mp));
        }
        ox[i] = rx;
        on[i] = rn;
      }
      const int64_t q0 = R0 + qr0;
      if constexpr (ARG) {
        T vx[V], vn[V];
        int64_t lx[V], ln[V];
#pragma unroll
        for (int i = 0; i < V; ++i) {
          vx[i] = ox[i].v;
          vn[i] = on[i].v;
          lx[i] = R0 + ox[i].i;
          ln[i] = R0 + on[i].i;
        }
        run_store<T>(s.omax ? s.omax + q0 : nullptr, s.omin ? s.omin + q0 : nullptr, ovec, dout, q0, R1, vx, vn);
        const int lmx = (int)(((uintptr_t)(amax + R0) / 8) & 1), lmn = (int)(((uintptr_t)(amin + R0) / 8) & 1);
        run_store<int64_t>(amax + q0, amin + q0, lmx == lmn, lmx, q0, R1, lx, ln);
      } else {
        run_store<T>(s.omax ? s.omax + q0 : nullptr, s.omin ? s.omin + q0 : nullptr, ovec, dout, q0, R1, ox, on);
      }
    }
#pragma unroll
    for (int i = 0; i < V; ++i) {
#pragma unroll
      for (int g = LAG - 1; g >= 1; --g) {
        hx[g][i] = hx[g - 1][i];
        hn[g][i] = hn[g - 1][i];
      }
      if (live) {
        hx[0][i] = ux[i];
        hn[0][i] = un[i];
      }
      cur[i] = nxt[i];
    }
    // Let this sub-tile's stores complete before the next one's loads are
    // issued: on MI355X 3-6% faster per launch than leaving them in flight
    // with the next loads at one or two sub-tiles of lag, even at four.  The
    // arg filter writes three times the bytes per output (values and 8-byte
    // locations) and gains from leaving them in flight while the next
    // sub-tile's scans run (n = 2^28 float32: w = 4096 2.33 -> 2.11 ms, w <=
    // 2048 1-2%); its next wait for loads then covers them.
    if constexpr (!ARG) __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0); expcnt, lgkmcnt untouched
    lds_barrier();  // ring slots of P_{k-1} may now be reused by P_{k+1}
  }
}

// Persistent: static round-robin over runs (runs share no data beyond a
// w-1 halo; on MI355X this beat the XCD-contiguous schedule by ~2%).
template <int MODE, class T, bool ARG = false, int LAG = 1>
__global__ __launch_bounds__(kTileThreads) void k_tile(Job<T> job) {
  __shared__ TileLds<typename ElemOf<T, ARG>::type, ARG && LAG == 1> sm;
  const int64_t nruns = job_tiles<MODE>(job);
  if constexpr (MODE == kJobDescs) {
    // Described series: workgroup g takes the g-th of gridDim.x equal,
    // contiguous ranges of the tiles (short ones: a sub-tile each) and
    // streams each series' part of it as one run.  One search finds the
    // range's first series; after that the walk only steps to the next
    // series, and a series' tiles in the range are never split into runs.
    const int64_t a = nruns * (int64_t)blockIdx.x / gridDim.x;
    const int64_t b = nruns * ((int64_t)blockIdx.x + 1) / gridDim.x;
    if (a >= b) return;
    int64_t k = find_series(job.pre, job.S, a);
    int64_t t = a, base = job.pre[k];
    while (t < b) {
      const int64_t next = job.pre[k + 1];  // k < S: pre[S] = nruns > t
      if (next > t) {
        const Series<T> s = job.descs[k];
        const int64_t nout = s.n - s.w + 1;
        const int64_t hi = min(b, next);
        run_body<T, ARG, LAG>(s, (t - base) * job.run, min(nout, (hi - base) * job.run), sm, job.amax, job.amin);
        t = hi;
      }
      base = next;
      ++k;
    }
    return;
  }
  for (int64_t t = blockIdx.x; t < nruns; t += gridDim.x) {
    int64_t local, gbase;
    const Series<T> s = job_series<MODE>(job, t, local, gbase);
    const int64_t nout = s.n - s.w + 1;
    const int64_t R0 = local * job.run;
    run_body<T, ARG, LAG>(s, R0, min(nout, R0 + job.run), sm, job.amax, job.amin);
  }
}

// =========================================================== chunk strategy
template <class T> struct ChunkLds {
  T xs[lds_len<T>(kChunkMax)];   // staged max outputs
  T hs[lds_len<T>(kChunkMax)];   // staged min outputs
  T red[4][kChunkThreads / 64];  // per-wave scan totals
  T dep[4];                      // PRE-side and SUF-side aggregates from look-back
  uint32_t ticket;
};

constexpr uint32_t kSpinLimit = 1u << 20;

// Aggregates live in a ring of 2^lg records indexed by the chunk's ticket;
// the tag mixes the launch epoch with the ring lap, so a record left by an
// earlier launch or an earlier lap never validates.
__device__ __forceinline__ uint64_t* ring_slot(const FlagRing& r, int64_t u) {
  return r.f + 4 * (u & ((int64_t(1) << r.lg) - 1));
}
__device__ __forceinline__ uint32_t ring_tag(const FlagRing& r, uint32_t ep, int64_t u) {
  uint32_t t = ep ^ ((uint32_t)(u >> r.lg) * 0x9E3779B1u);
  return t ? t : 0x80000000u;
}

// An aggregate record: 4 x 64-bit words, each (epoch << 32 | 32 payload
// bits).  Every word validates itself, so no fence orders them; readers
// and writers use agent-scope atomics, which stay coherent across XCDs.
template <class T> __device__ void publish(uint64_t* f, T mx, T mn, uint32_t ep) {
  const uint64_t e = (uint64_t)ep << 32;
  const uint64_t bx = to_bits(mx), bn = to_bits(mn);
  st_agent(f + 0, e | (bx & 0xFFFFFFFFull));
  st_agent(f + 2, e | (bn & 0xFFFFFFFFull));
  if constexpr (sizeof(T) == 8) {
    st_agent(f + 1, e | (bx >> 32));
    st_agent(f + 3, e | (bn >> 32));
  }
}

template <class T> __device__ void fetch(const uint64_t* f, uint32_t ep, T& mx, T& mn, Ctl* ctl) {
  uint64_t w0 = 0, w1 = 0, w2 = 0, w3 = 0;
  for (uint32_t spins = 0;; ++spins) {
    w0 = ld_agent(f + 0);
    w2 = ld_agent(f + 2);
    bool ok = (uint32_t)(w0 >> 32) == ep && (uint32_t)(w2 >> 32) == ep;
    if constexpr (sizeof(T) == 8) {
      w1 = ld_agent(f + 1);
      w3 = ld_agent(f + 3);
      ok = ok && (uint32_t)(w1 >> 32) == ep && (uint32_t)(w3 >> 32) == ep;
    }
    if (ok) break;
    if (spins >= kSpinLimit) {  // never expected: flag it for the host and move on
      st_agent32(&ctl->err, 1u);
      break;
    }
    __builtin_amdgcn_s_sleep(2);
  }
  const uint64_t bx = (w0 & 0xFFFFFFFFull) | ((w1 & 0xFFFFFFFFull) << 32);
  const uint64_t bn = (w2 & 0xFFFFFFFFull) | ((w3 & 0xFFFFFFFFull) << 32);
  mx = from_bits<T>(bx);
  mn = from_bits<T>(bn);
}

// Workgroup scan of two per-thread totals: exclusive prefix of (ax, an) in
// thread order and exclusive suffix of (bx, bn); also the inclusive total of
// (ax, an) over the workgroup.
template <class T, class Lds>
__device__ void wg_scan2(T& ax, T& an, T& bx, T& bn, T& tx, T& tn, Lds& sm) {
  constexpr int NW = kChunkThreads / 64;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  T ix = ax, in = an, jx = bx, jn = bn;
  wave_prefix2<T, true>(ix, in);
  wave_suffix2<T, true>(jx, jn);
  if (lane == 63) {
    sm.red[0][wave] = ix;
    sm.red[1][wave] = in;
  }
  if (lane == 0) {
    sm.red[2][wave] = jx;
    sm.red[3][wave] = jn;
  }
  __syncthreads();
  T cpx = Lim<T>::lo(), cpn = Lim<T>::hi(), csx = Lim<T>::lo(), csn = Lim<T>::hi();
  tx = Lim<T>::lo();
  tn = Lim<T>::hi();
#pragma unroll
  for (int v = 0; v < NW; ++v) {
    const T r0 = sm.red[0][v], r1 = sm.red[1][v], r2 = sm.red[2][v], r3 = sm.red[3][v];
    tx = hmax(tx, r0);
    tn = hmin(tn, r1);
    if (v < wave) {
      cpx = hmax(cpx, r0);
      cpn = hmin(cpn, r1);
    }
    if (v > wave) {
      csx = hmax(csx, r2);
      csn = hmin(csn, r3);
    }
  }
  T ex = shup(ix, 1, 64), en = shup(in, 1, 64), fx = shdn(jx, 1, 64), fn = shdn(jn, 1, 64);
  if (lane == 0) {
    ex = Lim<T>::lo();
    en = Lim<T>::hi();
  }
  if (lane == 63) {
    fx = Lim<T>::lo();
    fn = Lim<T>::hi();
  }
  ax = hmax(cpx, ex);
  an = hmin(cpn, en);
  bx = hmax(csx, fx);
  bn = hmin(csn, fn);
}

// Per-thread inputs of a chunk tile: own positions p0 + r and the shifted
// positions p0 - w + 1 + r of the chunk w back, r in [16*tid, 16*tid + 16).
template <class T>
__device__ __forceinline__ void chunk_load(const Series<T>& s, int64_t p0, int64_t w, int len, int lenfull, bool behind,
                                           T (&ax)[kChunkV], T (&an)[kChunkV], T (&bx)[kChunkV], T (&bn)[kChunkV]) {
  constexpr int V = kChunkV, EV = 16 / (int)sizeof(T);
  const int r0 = threadIdx.x * V;
  // fast path: one source segment, both ranges 16-byte aligned, full chunk
  const T* pa = nullptr;
  const int64_t lo = behind ? p0 - w : p0;
  if (p0 + len <= s.na) pa = s.a;
  else if (lo >= s.na) pa = s.b - s.na;
  const bool vec = pa != nullptr && len == lenfull && (lenfull % V) == 0 &&
                   ((((uintptr_t)(pa + p0)) | ((uintptr_t)(pa + lo))) & 15) == 0;
  if (vec) {
    T v[V];
    if (r0 < len) {
#pragma unroll
      for (int k = 0; k < V / EV; ++k) {
        const u32x4 u = gload((const u32x4*)(pa + p0 + r0 + k * EV));
        __builtin_memcpy(&v[k * EV], &u, 16);
      }
    }
#pragma unroll
    for (int i = 0; i < V; ++i) {
      const bool vo = r0 + i < len;
      ax[i] = vo ? v[i] : Lim<T>::lo();
      an[i] = vo ? v[i] : Lim<T>::hi();
    }
    if (behind) {
      // aligned load of a[p0-w+r0 .. +V) plus the element after: shift by one
      T u[V + 1];
      if (r0 < lenfull) {
#pragma unroll
        for (int k = 0; k < V / EV; ++k) {
          const u32x4 q = gload((const u32x4*)(pa + lo + r0 + k * EV));
          __builtin_memcpy(&u[k * EV], &q, 16);
        }
        u[V] = r0 + V < lenfull ? gload(pa + lo + r0 + V) : u[V - 1];
      }
#pragma unroll
      for (int i = 0; i < V; ++i) {
        const bool vb = r0 + i + 1 < lenfull;
        bx[i] = vb ? u[i + 1] : Lim<T>::lo();
        bn[i] = vb ? u[i + 1] : Lim<T>::hi();
      }
    } else {
#pragma unroll
      for (int i = 0; i < V; ++i) {
        bx[i] = Lim<T>::lo();
        bn[i] = Lim<T>::hi();
      }
    }
  } else {
#pragma unroll
    for (int i = 0; i < V; ++i) {
      const int r = r0 + i;
      const bool vo = r < len;
      const T x = vo ? src_at(s, p0 + r) : T(0);
      ax[i] = vo ? x : Lim<T>::lo();
      an[i] = vo ? x : Lim<T>::hi();
      const bool vb = behind && (r + 1 < lenfull);
      const T h = vb ? src_at(s, p0 - w + 1 + r) : T(0);
      bx[i] = vb ? h : Lim<T>::lo();
      bn[i] = vb ? h : Lim<T>::hi();
    }
  }
}

// Store staged outputs slots [rs, len) of buf to out[0 ..): lane-consecutive,
// 16-byte stores between a scalar head and tail.
template <class T>
__device__ __forceinline__ void chunk_store(T* out, const T* buf, int rs, int len) {
  constexpr int NT = kChunkThreads, EV = 16 / (int)sizeof(T);
  const int tid = threadIdx.x;
  int a0 = rs;
  while (a0 < len && (((uintptr_t)(out + a0)) & 15) != 0) ++a0;  // uniform, < EV steps
  for (int r = rs + tid; r < a0; r += NT) gstore(out + r, buf[lds_idx<T>(r)]);
  const int nv = (len - a0) / EV;
  for (int v = tid; v < nv; v += NT) {
    T e[EV];
#pragma unroll
    for (int k = 0; k < EV; ++k) e[k] = buf[lds_idx<T>(a0 + v * EV + k)];
    u32x4 u;
    __builtin_memcpy(&u, e, 16);
    gstore_nt((u32x4*)(out + a0 + v * EV), u);
  }
  for (int r = a0 + nv * EV + tid; r < len; r += NT) gstore(out + r, buf[lds_idx<T>(r)]);
}

// chunk_store of max(buf[r], c) (MAXF) or min(buf[r], c): a staged chunk's
// outputs with one more aggregate folded in as they leave LDS.
template <class T, bool MAXF>
__device__ __forceinline__ void chunk_store_fold(T* out, const T* buf, int rs, int len, T c) {
  constexpr int NT = kChunkThreads, EV = 16 / (int)sizeof(T);
  const int tid = threadIdx.x;
  auto f = [&](int r) { return MAXF ? hmax(buf[lds_idx<T>(r)], c) : hmin(buf[lds_idx<T>(r)], c); };
  int a0 = rs;
  while (a0 < len && (((uintptr_t)(out + a0)) & 15) != 0) ++a0;  // uniform, < EV steps
  for (int r = rs + tid; r < a0; r += NT) gstore(out + r, f(r));
  const int nv = (len - a0) / EV;
  for (int v = tid; v < nv; v += NT) {
    T e[EV];
#pragma unroll
    for (int k = 0; k < EV; ++k) e[k] = f(a0 + v * EV + k);
    u32x4 u;
    __builtin_memcpy(&u, e, 16);
    gstore_nt((u32x4*)(out + a0 + v * EV), u);
  }
  for (int r = a0 + nv * EV + tid; r < len; r += NT) gstore(out + r, f(r));
}

// counter: where the next ticket comes from.
template <class T>
__device__ void chunk_body(const Series<T>& s, int64_t t, int64_t gbase, const FlagRing& ring, uint32_t ep,
                           ChunkLds<T>& sm, Ctl* ctl, uint32_t* counter, uint32_t& next, bool warm = false) {
  constexpr int V = kChunkV;
  const int tid = threadIdx.x;
  const int64_t w = s.w, n = s.n;
  const int64_t K = (w + kChunkMax - 1) / kChunkMax;
  const int64_t C = (w + K - 1) / K;
  const int64_t b = t / K, k = t - b * K;
  const int64_t p0 = b * w + k * C;  // first input of the owned chunk
  const int lenfull = (int)min(C, w - k * C);
  const int len = (int)min((int64_t)lenfull, n - p0);
  // warm: a chunk just before this workgroup's ticket range, redone only to
  // publish its aggregate for the range's first chunks (no outputs)
  const bool behind = b >= 1 && !warm;
  const bool has_out = !warm && (p0 + len - 1) >= (w - 1);

  T ax[V], an[V], bx[V], bn[V];
  chunk_load<T>(s, p0, w, len, lenfull, behind, ax, an, bx, bn);

  // first look at the K-1 records this chunk depends on while the loads fly
  // (lane j of wave 0 reads chunk t-K+1+j); misses are re-read after publish
  const int64_t u0 = t - (K - 1);
  T fx = Lim<T>::lo(), fn = Lim<T>::hi();
  bool fok = true;
  if (has_out && tid < 64 && K - 1 <= 64) {
    const int64_t u = u0 + tid;
    if (u >= 0 && u < t) {
      const uint64_t* f = ring_slot(ring, gbase + u);
      const uint32_t tg = ring_tag(ring, ep, gbase + u);
      const uint64_t w0 = ld_agent(f + 0), w2 = ld_agent(f + 2);
      uint64_t w1 = 0, w3 = 0;
      fok = (uint32_t)(w0 >> 32) == tg && (uint32_t)(w2 >> 32) == tg;
      if constexpr (sizeof(T) == 8) {
        w1 = ld_agent(f + 1);
        w3 = ld_agent(f + 3);
        fok = fok && (uint32_t)(w1 >> 32) == tg && (uint32_t)(w3 >> 32) == tg;
      }
      fx = from_bits<T>((w0 & 0xFFFFFFFFull) | ((w1 & 0xFFFFFFFFull) << 32));
      fn = from_bits<T>((w2 & 0xFFFFFFFFull) | ((w3 & 0xFFFFFFFFull) << 32));
    }
  }

  if (s.carry != nullptr) {
    const int64_t cs = n - min(n, w - 1);
    const int r0 = tid * V;
#pragma unroll
    for (int i = 0; i < V; ++i)
      if (r0 + i < len && p0 + r0 + i >= cs) gstore(s.carry + (p0 + r0 + i - cs), ax[i]);
  }

#pragma unroll
  for (int i = 1; i < V; ++i) {
    ax[i] = hmax(ax[i - 1], ax[i]);
    an[i] = hmin(an[i - 1], an[i]);
  }
#pragma unroll
  for (int i = V - 2; i >= 0; --i) {
    bx[i] = hmax(bx[i + 1], bx[i]);
    bn[i] = hmin(bn[i + 1], bn[i]);
  }
  T epx = ax[V - 1], epn = an[V - 1], esx = bx[0], esn = bn[0], tx, tn;
  wg_scan2<T>(epx, epn, esx, esn, tx, tn, sm);
  // own chunk's aggregate, for the chunks after this one
  if (tid == 0) publish<T>(ring_slot(ring, gbase + t), tx, tn, ring_tag(ring, ep, gbase + t));

  if (has_out && tid < 64) {
    // (b, 0..k-1) feed PRE, (b-1, k+1..K-1) feed SUF
    T prx = Lim<T>::lo(), prn = Lim<T>::hi(), sux = Lim<T>::lo(), sun = Lim<T>::hi();
    for (int64_t base = u0; base < t; base += 64) {
      const int64_t u = base + tid;
      if (u >= 0 && u < t) {
        T mx = fx, mn = fn;
        if (!(base == u0 && K - 1 <= 64 && fok))
          fetch<T>(ring_slot(ring, gbase + u), ring_tag(ring, ep, gbase + u), mx, mn, ctl);
        if (u >= t - k) {
          prx = hmax(prx, mx);
          prn = hmin(prn, mn);
        } else {
          sux = hmax(sux, mx);
          sun = hmin(sun, mn);
        }
      }
    }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
      prx = hmax(prx, (T)__shfl_xor(prx, d, 64));
      prn = hmin(prn, (T)__shfl_xor(prn, d, 64));
      sux = hmax(sux, (T)__shfl_xor(sux, d, 64));
      sun = hmin(sun, (T)__shfl_xor(sun, d, 64));
    }
    if (tid == 0) {
      sm.dep[0] = prx;
      sm.dep[1] = prn;
      sm.dep[2] = sux;
      sm.dep[3] = sun;
    }
  }
  // Take the next ticket only now that this chunk waits on nothing: a ticket
  // taken earlier would sit unpublished behind this chunk's look-back and
  // stall the chunks that depend on it.  Its latency hides behind the stores.
  if (tid == 0) next = add_agent32(counter, 1u);
  __syncthreads();
  if (has_out) {
    const T prx = hmax(sm.dep[0], epx), prn = hmin(sm.dep[1], epn);
    const T sux = hmax(sm.dep[2], esx), sun = hmin(sm.dep[3], esn);
    // stage outputs: window ending at p0+r -> slot r
    const int r0 = tid * V;
#pragma unroll
    for (int i = 0; i < V; ++i) {
      const int r = r0 + i;
      if (r < len) {
        sm.xs[lds_idx<T>(r)] = hmax(hmax(bx[i], sux), hmax(prx, ax[i]));
        sm.hs[lds_idx<T>(r)] = hmin(hmin(bn[i], sun), hmin(prn, an[i]));
      }
    }
    __syncthreads();
    const int rs = (int)max((int64_t)0, (w - 1) - p0);  // first slot whose window starts at >= 0
    if (s.omax) chunk_store<T>(s.omax + (p0 - w + 1), sm.xs, rs, len);
    if (s.omin) chunk_store<T>(s.omin + (p0 - w + 1), sm.hs, rs, len);
  }
  __syncthreads();
}

// ================================================== long windows, two passes
// For a single series with K = ceil(w / 4096) > 1 chunks per block of w.
// Pass 1 (k_chunk_agg): every chunk's max and min.  Pass 2 (k_chunk_col):
// workgroup g walks column k = g mod K over a contiguous range of blocks;
// the chunk w back that each chunk's windows start in is the same column's
// previous chunk, which the workgroup loaded one step before and still
// holds in registers, and the aggregates of the chunks between come from
// pass 1.  Each input is read twice in all (once per pass) and nothing
// waits on another workgroup; the look-back kernel reads the chunk w back
// again from memory and waits on the records of the K-1 chunks before it.

// The raw inputs of chunk slots [r0, r0 + V) (slots >= len read as 0).
template <class T, int V>
__device__ __forceinline__ void col_load(const Series<T>& s, int64_t p0, int len, T (&v)[V]) {
  constexpr int EV = 16 / (int)sizeof(T);
  const int r0 = threadIdx.x * V;
  const T* pa = nullptr;
  if (p0 + len <= s.na) pa = s.a;
  else if (p0 >= s.na) pa = s.b - s.na;
  if (pa != nullptr && r0 + V <= len && (((uintptr_t)(pa + p0 + r0)) & 15) == 0) {
#pragma unroll
    for (int k = 0; k < V / EV; ++k) {
      const u32x4 u = gload((const u32x4*)(pa + p0 + r0 + k * EV));
      __builtin_memcpy(&v[k * EV], &u, 16);
    }
  } else {
#pragma unroll
    for (int i = 0; i < V; ++i) v[i] = r0 + i < len ? src_at(s, p0 + r0 + i) : T(0);
  }
}

// V: positions per thread, chunks of at most kChunkThreads * V inputs.
template <class T, int V>
__global__ __launch_bounds__(kChunkThreads) void k_chunk_agg(Series<T> s, T* aggx, T* aggn) {
  constexpr int64_t CM = int64_t(kChunkThreads) * V;
  __shared__ T red[2][kChunkThreads / 64];
  const int64_t w = s.w, n = s.n;
  const int64_t K = (w + CM - 1) / CM, C = (w + K - 1) / K;
  const int64_t nch = chunk_count(n, w, CM);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int64_t t = blockIdx.x; t < nch; t += gridDim.x) {
    const int64_t b = t / K, k = t - b * K;
    const int64_t p0 = b * w + k * C;
    const int len = (int)min(min(C, w - k * C), n - p0);
    T v[V];
    col_load<T, V>(s, p0, len, v);
    T mx = Lim<T>::lo(), mn = Lim<T>::hi();
#pragma unroll
    for (int i = 0; i < V; ++i)
      if ((int)threadIdx.x * V + i < len) {
        mx = hmax(mx, v[i]);
        mn = hmin(mn, v[i]);
      }
    for (int d = 32; d >= 1; d >>= 1) {
      mx = hmax(mx, (T)__shfl_xor(mx, d, 64));
      mn = hmin(mn, (T)__shfl_xor(mn, d, 64));
    }
    if (lane == 0) {
      red[0][wave] = mx;
      red[1][wave] = mn;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      T ax = red[0][0], an = red[1][0];
      for (int q = 1; q < kChunkThreads / 64; ++q) {
        ax = hmax(ax, red[0][q]);
        an = hmin(an, red[1][q]);
      }
      aggx[t] = ax;
      aggn[t] = an;
    }
    __syncthreads();
  }
}

template <class T, int V> struct ColLds {
  T xs[lds_len<T>(kChunkThreads * V)];  // staged max outputs
  T hs[lds_len<T>(kChunkThreads * V)];  // staged min outputs
  T red[4][kChunkThreads / 64];         // per-wave scan totals
  T dep[4];                             // PRE-side and SUF-side aggregates
};

template <class T, int V>
__global__ __launch_bounds__(kChunkThreads) void k_chunk_col(Series<T> s, const T* aggx, const T* aggn) {
  constexpr int64_t CM = int64_t(kChunkThreads) * V;
  __shared__ ColLds<T, V> sm;
  __shared__ T edge[kChunkThreads / 64];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t w = s.w, n = s.n;
  const int64_t K = (w + CM - 1) / CM, C = (w + K - 1) / K;
  const int64_t NB = (n + w - 1) / w;  // blocks, the last one partial
  const int64_t k = blockIdx.x % K, R = gridDim.x / K, rr = blockIdx.x / K;
  const int64_t per = (NB + R - 1) / R;
  const int64_t b0 = rr * per, b1 = min(NB, b0 + per);
  const int lenfull = (int)min(C, w - k * C);
  const int r0 = tid * V;
  T prev[V], cur[V];  // raw inputs of the column's previous chunk and of this one
  if (b0 >= b1 || b0 * w + k * C >= n) return;
  if (b0 >= 1) col_load<T, V>(s, (b0 - 1) * w + k * C, lenfull, prev);  // whole: it ends before block b0
  col_load<T, V>(s, b0 * w + k * C, (int)min((int64_t)lenfull, n - (b0 * w + k * C)), cur);
  for (int64_t b = b0; b < b1; ++b) {
    const int64_t p0 = b * w + k * C;
    if (p0 >= n) break;
    const int len = (int)min((int64_t)lenfull, n - p0);
    // the next chunk's loads fly while this one is computed
    T nxt[V];
    const int64_t p1 = p0 + w;
    if (b + 1 < b1 && p1 < n) col_load<T, V>(s, p1, (int)min((int64_t)lenfull, n - p1), nxt);
    // the aggregates this chunk needs, loaded now so their latency hides
    // behind the scans: (b, 0..k-1) feed PRE, (b-1, k+1..K-1) feed SUF
    const bool has_out = (p0 + len - 1) >= (w - 1);
    T gx0 = Lim<T>::lo(), gn0 = Lim<T>::hi(), gx1 = Lim<T>::lo(), gn1 = Lim<T>::hi();
    if (has_out && tid < 64) {
      for (int64_t j = tid; j < K; j += 64) {
        if (j < k) {
          gx0 = hmax(gx0, aggx[b * K + j]);
          gn0 = hmin(gn0, aggn[b * K + j]);
        } else if (j > k && b >= 1) {
          gx1 = hmax(gx1, aggx[(b - 1) * K + j]);
          gn1 = hmin(gn1, aggn[(b - 1) * K + j]);
        }
      }
    }
    if (s.carry != nullptr) {
      const int64_t cs = n - min(n, w - 1);
#pragma unroll
      for (int i = 0; i < V; ++i)
        if (r0 + i < len && p0 + r0 + i >= cs) gstore(s.carry + (p0 + r0 + i - cs), cur[i]);
    }
    // behind slot r: the previous chunk's slot r + 1 (the start of the
    // window that ends at slot r), from this lane, the next lane, or the
    // next wavefront's lane 0
    if (lane == 0) edge[wave] = prev[0];
    __syncthreads();
    T nb = __shfl_down(prev[0], 1, 64);
    if (lane == 63) nb = wave + 1 < kChunkThreads / 64 ? edge[wave + 1] : T(0);
    T ax[V], an[V], bx[V], bn[V];
    const bool behind = b >= 1;
#pragma unroll
    for (int i = 0; i < V; ++i) {
      const bool vo = r0 + i < len;
      ax[i] = vo ? cur[i] : Lim<T>::lo();
      an[i] = vo ? cur[i] : Lim<T>::hi();
      const bool vb = behind && r0 + i + 1 < lenfull;
      const T h = i + 1 < V ? prev[i + 1 < V ? i + 1 : 0] : nb;
      bx[i] = vb ? h : Lim<T>::lo();
      bn[i] = vb ? h : Lim<T>::hi();
    }
#pragma unroll
    for (int i = 1; i < V; ++i) {
      ax[i] = hmax(ax[i - 1], ax[i]);
      an[i] = hmin(an[i - 1], an[i]);
    }
#pragma unroll
    for (int i = V - 2; i >= 0; --i) {
      bx[i] = hmax(bx[i + 1], bx[i]);
      bn[i] = hmin(bn[i + 1], bn[i]);
    }
    T epx = ax[V - 1], epn = an[V - 1], esx = bx[0], esn = bn[0], tx, tn;
    wg_scan2<T>(epx, epn, esx, esn, tx, tn, sm);
    if (has_out && tid < 64) {
      T prx = gx0, prn = gn0, sux = gx1, sun = gn1;
#pragma unroll
      for (int d = 32; d >= 1; d >>= 1) {
        prx = hmax(prx, (T)__shfl_xor(prx, d, 64));
        prn = hmin(prn, (T)__shfl_xor(prn, d, 64));
        sux = hmax(sux, (T)__shfl_xor(sux, d, 64));
        sun = hmin(sun, (T)__shfl_xor(sun, d, 64));
      }
      if (tid == 0) {
        sm.dep[0] = prx;
        sm.dep[1] = prn;
        sm.dep[2] = sux;
        sm.dep[3] = sun;
      }
    }
    __syncthreads();
    if (has_out) {
      const T prx = hmax(sm.dep[0], epx), prn = hmin(sm.dep[1], epn);
      const T sux = hmax(sm.dep[2], esx), sun = hmin(sm.dep[3], esn);
#pragma unroll
      for (int i = 0; i < V; ++i) {
        const int r = r0 + i;
        if (r < len) {
          sm.xs[lds_idx<T>(r)] = hmax(hmax(bx[i], sux), hmax(prx, ax[i]));
          sm.hs[lds_idx<T>(r)] = hmin(hmin(bn[i], sun), hmin(prn, an[i]));
        }
      }
      __syncthreads();
      const int rs = (int)max((int64_t)0, (w - 1) - p0);  // first slot whose window starts at >= 0
      if (s.omax) chunk_store<T>(s.omax + (p0 - w + 1), sm.xs, rs, len);
      if (s.omin) chunk_store<T>(s.omin + (p0 - w + 1), sm.hs, rs, len);
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < V; ++i) {
      prev[i] = cur[i];
      cur[i] = nxt[i];
    }
  }
}

// One pass (k_chunk_col1): the same columns, without the aggregate pass.
// Each workgroup publishes its chunk's max and min (a tagged record, as the
// look-back kernel's) as soon as its scans give them, and reads the chunks
// between from its siblings' records: (b, 0..k-1) are published by the
// range's other workgroups in the same step, (b-1, k+1..K-1) one step
// earlier.  A range's first block needs the block before it, which the
// previous range reaches only at its end, so every workgroup also publishes
// its column's chunk of that block (loaded anyway; the previous range later
// publishes the same values).  DEFER: a chunk's outputs wait one step for
// the siblings' records -- at step b a workgroup stages everything it knows
// of chunk b's windows (its own prefix and the previous chunk's suffix,
// across the workgroup) in LDS, and only after publishing chunk b+1 fetches
// the records chunk b needs and stores its outputs with them folded in, so
// the K workgroups of a range do not wait on each other's current step.
// On MI355X (n = 2^28) that pays where K is large (float32 w = 262144, K =
// 64: 0.81 -> 0.75 ms; 2^20, K = 256: 0.89 -> 0.79; float64 w = 65536, K =
// 32: 1.51 -> 1.40) and costs 3-6% where it is small (float32 w = 8193 ..
// 65536, K <= 16: 0.78 -> 0.81 ms at 65536), so it is taken from K = 32.  A
// workgroup publishes before it waits, and waits only on records of its own
// step or earlier, so with every workgroup resident (the launch is
// cooperative) every wait ends; one that outlasts the spin limit sets the
// error word instead of hanging.
template <class T, int V, bool DEFER>
__global__ __launch_bounds__(kChunkThreads) void k_chunk_col1(Series<T> s, uint64_t* rec, Ctl* ctl) {
  constexpr int64_t CM = int64_t(kChunkThreads) * V;
  constexpr int NW = kChunkThreads / 64;
  __shared__ ColLds<T, V> sm;
  __shared__ T edge[NW];
  __shared__ T pro[2][NW];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t w = s.w, n = s.n;
  const int64_t K = (w + CM - 1) / CM, C = (w + K - 1) / K;
  const int64_t NB = (n + w - 1) / w;  // blocks, the last one partial
  const int64_t k = blockIdx.x % K, R = gridDim.x / K, rr = blockIdx.x / K;
  const int64_t per = (NB + R - 1) / R;
  const int64_t b0 = rr * per, b1 = min(NB, b0 + per);
  const int lenfull = (int)min(C, w - k * C);
  const int r0 = tid * V;
  const uint32_t ep = ld_agent32(&ctl->epoch);
  T prev[V], cur[V];  // raw inputs of the column's previous chunk and of this one
  if (b0 < b1) {
    // (published also when this column has no chunk in block b0: a sibling
    // with one may need it)
    if (b0 >= 1) {
      col_load<T, V>(s, (b0 - 1) * w + k * C, lenfull, prev);  // whole: it ends before block b0
      T mx = Lim<T>::lo(), mn = Lim<T>::hi();
#pragma unroll
      for (int i = 0; i < V; ++i)
        if (r0 + i < lenfull) {
          mx = hmax(mx, prev[i]);
          mn = hmin(mn, prev[i]);
        }
      for (int d = 32; d >= 1; d >>= 1) {
        mx = hmax(mx, (T)__shfl_xor(mx, d, 64));
        mn = hmin(mn, (T)__shfl_xor(mn, d, 64));
      }
      if (lane == 0) {
        pro[0][wave] = mx;
        pro[1][wave] = mn;
      }
      __syncthreads();
      if (tid == 0) {
        for (int q = 1; q < NW; ++q) {
          mx = hmax(mx, pro[0][q]);
          mn = hmin(mn, pro[1][q]);
        }
        publish<T>(rec + 4 * ((b0 - 1) * K + k), mx, mn, ep);
      }
    }
  }
  // Stores of chunk (b, k), staged in LDS a step earlier: fold in the
  // siblings' chunks (b, 0..k-1) on the PRE side and (b-1, k+1..K-1) on the
  // SUF side, then write the outputs; the LDS is free again on return.
  auto flush = [&](int64_t b) {
    const int64_t p0 = b * w + k * C;
    const int len = (int)min((int64_t)lenfull, n - p0);
    if (tid < 64) {
      T ax = Lim<T>::lo(), an = Lim<T>::hi();
      for (int64_t j = tid; j < K; j += 64) {
        if (j < k || (j > k && b >= 1)) {
          T mx, mn;
          fetch<T>(rec + 4 * ((j < k ? b : b - 1) * K + j), ep, mx, mn, ctl);
          ax = hmax(ax, mx);
          an = hmin(an, mn);
        }
      }
#pragma unroll
      for (int d = 32; d >= 1; d >>= 1) {
        ax = hmax(ax, (T)__shfl_xor(ax, d, 64));
        an = hmin(an, (T)__shfl_xor(an, d, 64));
      }
      if (tid == 0) {
        sm.dep[0] = ax;
        sm.dep[1] = an;
      }
    }
    __syncthreads();
    const int rs = (int)max((int64_t)0, (w - 1) - p0);  // first slot whose window starts at >= 0
    if (s.omax) chunk_store_fold<T, true>(s.omax + (p0 - w + 1), sm.xs, rs, len, sm.dep[0]);
    if (s.omin) chunk_store_fold<T, false>(s.omin + (p0 - w + 1), sm.hs, rs, len, sm.dep[1]);
    __syncthreads();
  };
  bool pend = false;  // a chunk's outputs wait in LDS for its siblings' records
  int64_t pb = 0;     // its block
  if (b0 < b1 && b0 * w + k * C < n) {
    col_load<T, V>(s, b0 * w + k * C, (int)min((int64_t)lenfull, n - (b0 * w + k * C)), cur);
    for (int64_t b = b0; b < b1; ++b) {
      const int64_t p0 = b * w + k * C;
      if (p0 >= n) break;
      const int len = (int)min((int64_t)lenfull, n - p0);
      // the next chunk's loads fly while this one is computed
      T nxt[V];
      const int64_t p1 = p0 + w;
      if (b + 1 < b1 && p1 < n) col_load<T, V>(s, p1, (int)min((int64_t)lenfull, n - p1), nxt);
      const bool has_out = (p0 + len - 1) >= (w - 1);
      if (s.carry != nullptr) {
        const int64_t cs = n - min(n, w - 1);
#pragma unroll
        for (int i = 0; i < V; ++i)
          if (r0 + i < len && p0 + r0 + i >= cs) gstore(s.carry + (p0 + r0 + i - cs), cur[i]);
      }
      // behind slot r: the previous chunk's slot r + 1 (the start of the
      // window that ends at slot r), from this lane, the next lane, or the
      // next wavefront's lane 0
      if (lane == 0) edge[wave] = prev[0];
      __syncthreads();
      T nb = __shfl_down(prev[0], 1, 64);
      if (lane == 63) nb = wave + 1 < NW ? edge[wave + 1] : T(0);
      T ax[V], an[V], bx[V], bn[V];
      const bool behind = b >= 1;
#pragma unroll
      for (int i = 0; i < V; ++i) {
        const bool vo = r0 + i < len;
        ax[i] = vo ? cur[i] : Lim<T>::lo();
        an[i] = vo ? cur[i] : Lim<T>::hi();
        const bool vb = behind && r0 + i + 1 < lenfull;
        const T h = i + 1 < V ? prev[i + 1 < V ? i + 1 : 0] : nb;
        bx[i] = vb ? h : Lim<T>::lo();
        bn[i] = vb ? h : Lim<T>::hi();
      }
#pragma unroll
      for (int i = 1; i < V; ++i) {
        ax[i] = hmax(ax[i - 1], ax[i]);
        an[i] = hmin(an[i - 1], an[i]);
      }
#pragma unroll
      for (int i = V - 2; i >= 0; --i) {
        bx[i] = hmax(bx[i + 1], bx[i]);
        bn[i] = hmin(bn[i + 1], bn[i]);
      }
      T epx = ax[V - 1], epn = an[V - 1], esx = bx[0], esn = bn[0], tx, tn;
      wg_scan2<T>(epx, epn, esx, esn, tx, tn, sm);
      // this chunk's max and min, for the siblings' windows
      if (tid == 0) publish<T>(rec + 4 * (b * K + k), tx, tn, ep);
      if constexpr (DEFER) {
        // the previous step's chunk: its siblings' records, then its outputs
        if (pend) flush(pb);
        if (has_out) {
          // what this workgroup knows of the windows ending in this chunk:
          // the previous chunk's suffix and this one's prefix, each completed
          // across the workgroup (the siblings' chunks come a step later)
#pragma unroll
          for (int i = 0; i < V; ++i) {
            const int r = r0 + i;
            if (r < len) {
              sm.xs[lds_idx<T>(r)] = hmax(hmax(bx[i], esx), hmax(epx, ax[i]));
              sm.hs[lds_idx<T>(r)] = hmin(hmin(bn[i], esn), hmin(epn, an[i]));
            }
          }
        }
        pend = has_out;
        pb = b;
      } else {
        if (has_out && tid < 64) {
          // (b, 0..k-1) feed PRE, (b-1, k+1..K-1) feed SUF
          T prx = Lim<T>::lo(), prn = Lim<T>::hi(), sux = Lim<T>::lo(), sun = Lim<T>::hi();
          for (int64_t j = tid; j < K; j += 64) {
            if (j < k) {
              T mx, mn;
              fetch<T>(rec + 4 * (b * K + j), ep, mx, mn, ctl);
              prx = hmax(prx, mx);
              prn = hmin(prn, mn);
            } else if (j > k && b >= 1) {
              T mx, mn;
              fetch<T>(rec + 4 * ((b - 1) * K + j), ep, mx, mn, ctl);
              sux = hmax(sux, mx);
              sun = hmin(sun, mn);
            }
          }
#pragma unroll
          for (int d = 32; d >= 1; d >>= 1) {
            prx = hmax(prx, (T)__shfl_xor(prx, d, 64));
            prn = hmin(prn, (T)__shfl_xor(prn, d, 64));
            sux = hmax(sux, (T)__shfl_xor(sux, d, 64));
            sun = hmin(sun, (T)__shfl_xor(sun, d, 64));
          }
          if (tid == 0) {
            sm.dep[0] = prx;
            sm.dep[1] = prn;
            sm.dep[2] = sux;
            sm.dep[3] = sun;
          }
        }
        __syncthreads();
        if (has_out) {
          const T prx = hmax(sm.dep[0], epx), prn = hmin(sm.dep[1], epn);
          const T sux = hmax(sm.dep[2], esx), sun = hmin(sm.dep[3], esn);
#pragma unroll
          for (int i = 0; i < V; ++i) {
            const int r = r0 + i;
            if (r < len) {
              sm.xs[lds_idx<T>(r)] = hmax(hmax(bx[i], sux), hmax(prx, ax[i]));
              sm.hs[lds_idx<T>(r)] = hmin(hmin(bn[i], sun), hmin(prn, an[i]));
            }
          }
          __syncthreads();
          const int rs = (int)max((int64_t)0, (w - 1) - p0);  // first slot whose window starts at >= 0
          if (s.omax) chunk_store<T>(s.omax + (p0 - w + 1), sm.xs, rs, len);
          if (s.omin) chunk_store<T>(s.omin + (p0 - w + 1), sm.hs, rs, len);
        }
      }
      __syncthreads();
#pragma unroll
      for (int i = 0; i < V; ++i) {
        prev[i] = cur[i];
        cur[i] = nxt[i];
      }
    }
    if constexpr (DEFER)
      if (pend) flush(pb);
  }
  // the last workgroup out bumps the epoch (no record of this launch
  // validates in the next one)
  if (tid == 0) {
    const uint32_t d = add_agent32(&ctl->done, 1u);
    if (d == gridDim.x - 1) {
      st_agent32(&ctl->done, 0u);
      uint32_t e = ep + 1u;
      if (e == 0u) e = 1u;
      st_agent32(&ctl->epoch, e);
    }
  }
}

template <int MODE, class T>
__global__ __launch_bounds__(kChunkThreads) void k_chunk(Job<T> job) {
  __shared__ ChunkLds<T> sm;
  Ctl* ctl = job.ctl;
  const int64_t ntiles = job_tiles<MODE>(job);
  // no chunks (a batch with no long window): touch no control word, so the
  // next launch finds them as this one did (no records were published)
  if (ntiles == 0) return;
  const uint32_t ep = ld_agent32(&ctl->epoch);
  // A single series may split into R contiguous ranges of chunks, each with
  // its own in-order tickets and served by the workgroups with blockIdx % R
  // equal to its number.  Workgroup ids go round robin over the 8 XCDs, so
  // with R a multiple of 8 a range stays on one XCD, and the chunk w back
  // that each chunk re-reads was loaded there a moment earlier and is still
  // in that XCD's L2.  The placement matters for speed only.  With K > 1 a
  // range first redoes the K-1 chunks before it (loads and publishes their
  // aggregates, identical to what the range before publishes), so its first
  // chunks wait only on its own workgroups; this needs every chunk of the
  // launch to own a ring slot.
  const int R = MODE == kJobOne ? job.ranges : 0;
  const int64_t K1 = MODE == kJobOne ? (job.one.w + kChunkMax - 1) / kChunkMax : 1;
  const bool split = R > 1 && ntiles >= 32 * (int64_t)R && (int)gridDim.x >= 8 * R && K1 <= 64 &&
                     (K1 == 1 || ntiles <= (int64_t(1) << job.ring.lg));
  const int cls = split ? (int)(blockIdx.x % R) : 0;
  const int64_t rlo = split ? ntiles * cls / R : 0, rhi = split ? ntiles * (cls + 1) / R : ntiles;
  const int64_t rfirst = split ? max((int64_t)0, rlo - (K1 - 1)) : 0;  // first ticketed chunk
  uint32_t* counter = split ? &ctl->tick[cls][0] : &ctl->ticket;
  // thread 0 takes each next ticket while the current chunk stores its outputs
  uint32_t next = 0;
  if (threadIdx.x == 0) next = add_agent32(counter, 1u);
  for (;;) {
    if (threadIdx.x == 0) sm.ticket = next;
    __syncthreads();
    const int64_t t = rfirst + (int64_t)sm.ticket;
    if (t >= rhi) break;
    int64_t local, gbase;
    const Series<T> s = job_series<MODE>(job, t, local, gbase);
    chunk_body<T>(s, local, gbase, job.ring, ep, sm, ctl, counter, next, t < rlo);
  }
  // the last workgroup out re-arms the control words for the next launch
  if (threadIdx.x == 0) {
    const uint32_t d = add_agent32(&ctl->done, 1u);
    if (d == gridDim.x - 1) {
      st_agent32(&ctl->ticket, 0u);
      for (int i = 0; i < R && i < kMaxRanges; ++i) st_agent32(&ctl->tick[i][0], 0u);
      st_agent32(&ctl->done, 0u);
      uint32_t e = ep + 1u;
      if (e == 0u) e = 1u;
      st_agent32(&ctl->epoch, e);
    }
  }
}

// ================================================ arg filter, long windows
// A window [j, j+p) is the union of the F windows of a shorter length q
// starting at j, j+q, ..., j+(F-2)q and j+p-q when p <= F q (they overlap
// at the end), so its leftmost max (min) is the leftmost of their (value,
// location) results.  One step maps window q's outputs to window p's; long
// windows start from a tile-kernel pass (w > kTileMaxW).  The F reads of an
// output hit consecutive addresses across a wavefront and mostly come from
// cache.
template <class T>
__global__ __launch_bounds__(256) void k_argcombine(const T* __restrict__ vx, const T* __restrict__ vn,
                                                    const int64_t* __restrict__ ix, const int64_t* __restrict__ in_,
                                                    int64_t q, int64_t p, int F, int64_t nout, T* __restrict__ ox,
                                                    T* __restrict__ on, int64_t* __restrict__ jx,
                                                    int64_t* __restrict__ jn) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < nout; j += stride) {
    T bx = gload(vx + j), bn = gload(vn + j);
    int64_t lx = gload(ix + j), ln = gload(in_ + j);
    for (int f = 1; f < F; ++f) {
      const int64_t o = j + min((int64_t)f * q, p - q);
      const T a = gload(vx + o), c = gload(vn + o);
      const int64_t la = gload(ix + o), lc = gload(in_ + o);
      // equal values: the smaller location wins (all lie in the window)
      if (a > bx || (a == bx && la < lx)) {
        bx = a;
        lx = la;
      }
      if (c < bn || (c == bn && lc < ln)) {
        bn = c;
        ln = lc;
      }
    }
    gstore(ox + j, bx);
    gstore(jx + j, lx);
    gstore(on + j, bn);
    gstore(jn + j, ln);
  }
}

// ==================================================== centered envelopes
// Envelope of radius r: upper[i] / lower[i] = max / min over
// [max(0, i-r), min(n-1, i+r)] (windows truncated at the series ends; the
// time-warping lower bound the paper cites in Section 1).  The interior
// i in [r, n-1-r] is the valid filter of width 2r+1, written by the 1-D
// kernels at offset r; these kernels write the two truncated ends.  One
// workgroup scans an end (the first or the last min(n, 2r) elements) in
// tiles of 2048 with a running carry: scan index k (position k from the
// left, or n-1-k from the right) gives the output at k-r (left) or
// n-1-k+r (right) once k >= r.  When n <= 2r the left scan reaches the last
// element and its total is the envelope of every window truncated at both
// ends.
template <class T>
__device__ void env_end(const T* a, int64_t n, int64_t r, T* up, T* lo, bool left, T* sx, T* sn) {
  constexpr int V = 8, NT = 256, TT = NT * V;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int64_t m = min(n, 2 * r);
  T cx = Lim<T>::lo(), cn = Lim<T>::hi();  // over the tiles already scanned
  for (int64_t base = 0; base < m; base += TT) {
    T px[V], pn[V];
    T rx = Lim<T>::lo(), rn = Lim<T>::hi();
#pragma unroll
    for (int i = 0; i < V; ++i) {
      const int64_t k = base + tid * V + i;
      if (k < m) {
        const T v = gload(a + (left ? k : n - 1 - k));
        rx = vmax(rx, v);
        rn = vmin(rn, v);
      }
      px[i] = rx;
      pn[i] = rn;
    }
    // exclusive prefix of the thread totals: lanes, then waves
    T ix = rx, in = rn;
    wave_prefix2(ix, in);
    T ex = shup(ix, 1, 64), en = shup(in, 1, 64);
    if (lane == 0) {
      ex = Lim<T>::lo();
      en = Lim<T>::hi();
    }
    if (lane == 63) {
      sx[wv] = ix;
      sn[wv] = in;
    }
    __syncthreads();
    T wx = Lim<T>::lo(), wn = Lim<T>::hi(), tx = Lim<T>::lo(), tn = Lim<T>::hi();
#pragma unroll
    for (int v = 0; v < NT / 64; ++v) {
      if (v < wv) {
        wx = vmax(wx, sx[v]);
        wn = vmin(wn, sn[v]);
      }
      tx = vmax(tx, sx[v]);
      tn = vmin(tn, sn[v]);
    }
    __syncthreads();  // sx / sn are rewritten by the next tile
    const T ox = vmax(cx, vmax(wx, ex)), on = vmin(cn, vmin(wn, en));
#pragma unroll
    for (int i = 0; i < V; ++i) {
      const int64_t k = base + tid * V + i;
      if (k < m && k >= r) {
        const int64_t o = left ? k - r : n - 1 - k + r;
        gstore(up + o, vmax(ox, px[i]));
        gstore(lo + o, vmin(on, pn[i]));
      }
    }
    cx = vmax(cx, tx);
    cn = vmin(cn, tn);
  }
  if (left && m == n) {
    // windows truncated at both ends: the whole series
    for (int64_t i = max((int64_t)0, n - r) + tid; i < min(r, n); i += NT) {
      gstore(up + i, cx);
      gstore(lo + i, cn);
    }
  }
}

// blockIdx.x: 0 the left end, 1 the right end
template <class T>
__global__ __launch_bounds__(256) void k_env_ends(const T* a, int64_t n, int64_t r, T* up, T* lo) {
  __shared__ T sx[4], sn[4];
  env_end<T>(a, n, r, up, lo, blockIdx.x == 0, sx, sn);
}

// The same end scan by one wavefront (no barriers), for the many short ends
// of a batch: passes of 512 elements with a running carry.
template <class T>
__device__ void env_end_wave(const T* a, int64_t n, int64_t r, T* up, T* lo, bool left) {
  constexpr int V = 8, WT = 64 * V;
  const int lane = threadIdx.x & 63;
  const int64_t m = min(n, 2 * r);
  T cx = Lim<T>::lo(), cn = Lim<T>::hi();
  for (int64_t base = 0; base < m; base += WT) {
    T px[V], pn[V];
    T rx = Lim<T>::lo(), rn = Lim<T>::hi();
#pragma unroll
    for (int i = 0; i < V; ++i) {
      const int64_t k = base + lane * V + i;
      if (k < m) {
        const T v = gload(a + (left ? k : n - 1 - k));
        rx = vmax(rx, v);
        rn = vmin(rn, v);
      }
      px[i] = rx;
      pn[i] = rn;
    }
    T ix = rx, in = rn;
    wave_prefix2(ix, in);
    T ex = shup(ix, 1, 64), en = shup(in, 1, 64);
    if (lane == 0) {
      ex = Lim<T>::lo();
      en = Lim<T>::hi();
    }
    const T tx = readlane(ix, 63), tn = readlane(in, 63);
    const T ox = vmax(cx, ex), on = vmin(cn, en);
#pragma unroll
    for (int i = 0; i < V; ++i) {
      const int64_t k = base + lane * V + i;
      if (k < m && k >= r) {
        const int64_t o = left ? k - r : n - 1 - k + r;
        gstore(up + o, vmax(ox, px[i]));
        gstore(lo + o, vmin(on, pn[i]));
      }
    }
    cx = vmax(cx, tx);
    cn = vmin(cn, tn);
  }
  if (left && m == n) {
    for (int64_t i = max((int64_t)0, n - r) + lane; i < min(r, n); i += 64) {
      gstore(up + i, cx);
      gstore(lo + i, cn);
    }
  }
}

// one wavefront per series end: end e = global wave id, series e / 2, side
// e % 2 (0 left, 1 right)
template <class T>
__global__ __launch_bounds__(256) void k_env_ends_batched(const T* in, const int64_t* off, const int64_t* radii,
                                                          int64_t S, T* up, T* lo) {
  const int64_t nw = (int64_t)gridDim.x * (blockDim.x / 64);
  for (int64_t e = (int64_t)blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6); e < 2 * S; e += nw) {
    const int64_t k = e >> 1;
    const int64_t s0 = off[k], n = off[k + 1] - s0, r = radii[k];
    if (r > 0 && n > 0 && !env_short(n, r)) env_end_wave<T>(in + s0, n, r, up + s0, lo + s0, (e & 1) == 0);
  }
}

// Batched envelope interiors as a batched filter: window 2r+1, outputs at
// the series' own offset + r.  A negative radius gives a window < 1, which
// the batched filter skips.
__global__ __launch_bounds__(256) void k_env_setup(const int64_t* off, const int64_t* radii, int64_t S, int64_t* wins,
                                                    int64_t* oo) {
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k <= S; k += (int64_t)gridDim.x * blockDim.x) {
    if (k < S) {
      const int64_t n = off[k + 1] - off[k];
      // a short series is served whole by k_env_short: no window here
      wins[k] = env_short(n, radii[k]) ? n + 1 : 2 * radii[k] + 1;
      oo[k] = off[k] + radii[k];
    } else {
      oo[k] = off[k];
    }
  }
}

// ============================================ chunk runs (local aggregates)
// Same window-aligned chunks as above (at most kCrMax inputs), but a
// workgroup walks a run of consecutive chunks of one series and keeps the
// aggregates of the last chunks in an LDS ring, so nothing is shared between
// workgroups: no tickets, no look-back.  A run first reduces the K-1 chunks
// before it (a warm-up read of about w inputs); the planner uses this kernel
// only where that extra read is small against the run.  The next chunk's
// loads are issued before the current chunk is computed.
template <class T> struct CrunLds {
  T xs[lds_len<T>(kCrMax)];  // staged max outputs
  T hs[lds_len<T>(kCrMax)];  // staged min outputs
  T red[4][kChunkThreads / 64];
  T dep[4];
  T agx[kCrRing];  // chunk aggregates, indexed by chunk mod kCrRing
  T agn[kCrRing];
};

// Raw inputs of chunk c for this thread: own positions p0 + r and shifted
// positions p0 - w + 1 + r of the chunk w back, r in [8*tid, 8*tid + 8).
// Positions outside the chunk read as 0 and are masked later.
template <class T>
__device__ __forceinline__ void crun_raw(const Series<T>& s, int64_t p0, int64_t w, int len, int lenfull, bool behind,
                                         T (&own)[kCrV], T (&beh)[kCrV]) {
  constexpr int V = kCrV, EV = 16 / (int)sizeof(T);
  const int r0 = threadIdx.x * V;
  const T* pa = nullptr;
  const int64_t lo = behind ? p0 - w : p0;
  if (p0 + len <= s.na) pa = s.a;
  else if (lo >= s.na) pa = s.b - s.na;
  const bool vec = pa != nullptr && len == lenfull && (lenfull % V) == 0 &&
                   ((((uintptr_t)(pa + p0)) | ((uintptr_t)(pa + lo))) & 15) == 0;
  if (vec) {
    if (r0 < len) {
#pragma unroll
      for (int k = 0; k < V / EV; ++k) {
        const u32x4 u = gload((const u32x4*)(pa + p0 + r0 + k * EV));
        __builtin_memcpy(&own[k * EV], &u, 16);
      }
    }
    if (behind && r0 < lenfull) {
      T u[V + 1];
#pragma unroll
      for (int k = 0; k < V / EV; ++k) {
        const u32x4 q = gload((const u32x4*)(pa + lo + r0 + k * EV));
        __builtin_memcpy(&u[k * EV], &q, 16);
      }
      u[V] = r0 + V < lenfull ? gload(pa + lo + r0 + V) : T(0);
#pragma unroll
      for (int i = 0; i < V; ++i) beh[i] = u[i + 1];
    }
  } else {
#pragma unroll
    for (int i = 0; i < V; ++i) {
      const int r = r0 + i;
      own[i] = r < len ? src_at(s, p0 + r) : T(0);
      beh[i] = (behind && r + 1 < lenfull) ? src_at(s, p0 - w + 1 + r) : T(0);
    }
  }
}

template <class T>
__device__ void crun_body(const Series<T>& s, int64_t c0, int64_t c1, CrunLds<T>& sm) {
  constexpr int V = kCrV;
  const int tid = threadIdx.x;
  const int64_t w = s.w, n = s.n;
  const int64_t K = (w + kCrMax - 1) / kCrMax;
  const int64_t C = (w + K - 1) / K;
  const int64_t cw = max((int64_t)0, c0 - (K - 1));  // warm-up: aggregates only
  const int r0 = tid * V;
  T own[V], beh[V], nown[V], nbeh[V];
  auto geom = [&](int64_t c, int64_t& p0, int& lenfull, int& len) {
    const int64_t b = c / K, k = c - b * K;
    p0 = b * w + k * C;
    lenfull = (int)min(C, w - k * C);
    len = (int)min((int64_t)lenfull, n - p0);
  };
  {
    int64_t p0;
    int lf, ln;
    geom(cw, p0, lf, ln);
    crun_raw<T>(s, p0, w, ln, lf, cw >= c0 && p0 >= w, own, beh);
  }
  for (int64_t c = cw; c < c1; ++c) {
    int64_t p0;
    int lenfull, len;
    geom(c, p0, lenfull, len);
    const int64_t b = c / K, k = c - b * K;
    const bool work = c >= c0;
    const bool behind = work && b >= 1;
    if (c + 1 < c1) {
      int64_t q0;
      int lf, ln;
      geom(c + 1, q0, lf, ln);
      crun_raw<T>(s, q0, w, ln, lf, c + 1 >= c0 && q0 >= w, nown, nbeh);
    }
    T ax[V], an[V], bx[V], bn[V];
#pragma unroll
    for (int i = 0; i < V; ++i) {
      const int r = r0 + i;
      const bool vo = r < len;
      ax[i] = vo ? own[i] : Lim<T>::lo();
      an[i] = vo ? own[i] : Lim<T>::hi();
      const bool vb = behind && (r + 1 < lenfull);
      bx[i] = vb ? beh[i] : Lim<T>::lo();
      bn[i] = vb ? beh[i] : Lim<T>::hi();
    }
    if (work && s.carry != nullptr) {
      const int64_t cs = n - min(n, w - 1);
#pragma unroll
      for (int i = 0; i < V; ++i)
        if (r0 + i < len && p0 + r0 + i >= cs) gstore(s.carry + (p0 + r0 + i - cs), own[i]);
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
    T epx = ax[V - 1], epn = an[V - 1], esx = bx[0], esn = bn[0], tx, tn;
    wg_scan2<T>(epx, epn, esx, esn, tx, tn, sm);
    if (tid == 0) {
      sm.agx[c & (kCrRing - 1)] = tx;
      sm.agn[c & (kCrRing - 1)] = tn;
    }
    const bool has_out = work && (p0 + len - 1) >= (w - 1);
    if (has_out && tid < 64) {
      // (b, 0..k-1) feed PRE, (b-1, k+1..K-1) feed SUF: all in the ring
      T prx = Lim<T>::lo(), prn = Lim<T>::hi(), sux = Lim<T>::lo(), sun = Lim<T>::hi();
      for (int64_t u = c - (K - 1) + tid; u < c; u += 64) {
        if (u >= 0) {
          const T mx = sm.agx[u & (kCrRing - 1)], mn = sm.agn[u & (kCrRing - 1)];
          if (u >= c - k) {
            prx = vmax(prx, mx);
            prn = vmin(prn, mn);
          } else {
            sux = vmax(sux, mx);
            sun = vmin(sun, mn);
          }
        }
      }
#pragma unroll
      for (int d = 32; d >= 1; d >>= 1) {
        prx = vmax(prx, (T)__shfl_xor(prx, d, 64));
        prn = vmin(prn, (T)__shfl_xor(prn, d, 64));
        sux = vmax(sux, (T)__shfl_xor(sux, d, 64));
        sun = vmin(sun, (T)__shfl_xor(sun, d, 64));
      }
      if (tid == 0) {
        sm.dep[0] = prx;
        sm.dep[1] = prn;
        sm.dep[2] = sux;
        sm.dep[3] = sun;
      }
    }
    __syncthreads();
    if (has_out) {
      const T prx = vmax(sm.dep[0], epx), prn = vmin(sm.dep[1], epn);
      const T sux = vmax(sm.dep[2], esx), sun = vmin(sm.dep[3], esn);
#pragma unroll
      for (int i = 0; i < V; ++i) {
        const int r = r0 + i;
        if (r < len) {
          sm.xs[lds_idx<T>(r)] = vmax(vmax(bx[i], sux), vmax(prx, ax[i]));
          sm.hs[lds_idx<T>(r)] = vmin(vmin(bn[i], sun), vmin(prn, an[i]));
        }
      }
      __syncthreads();
      const int rs = (int)max((int64_t)0, (w - 1) - p0);
      if (s.omax) chunk_store<T>(s.omax + (p0 - w + 1), sm.xs, rs, len);
      if (s.omin) chunk_store<T>(s.omin + (p0 - w + 1), sm.hs, rs, len);
    }
#pragma unroll
    for (int i = 0; i < V; ++i) {
      own[i] = nown[i];
      beh[i] = nbeh[i];
    }
    __syncthreads();
  }
}

// Persistent: XCD-aware static schedule over runs of `job.run` chunks.
template <int MODE, class T>
__global__ __launch_bounds__(kChunkThreads) void k_crun(Job<T> job) {
  __shared__ CrunLds<T> sm;
  const int64_t nruns = job_tiles<MODE>(job);
  int64_t first, stride, end;
  xcd_schedule(nruns, first, stride, end);
  for (int64_t t = first; t < end; t += stride) {
    int64_t local, gbase;
    const Series<T> s = job_series<MODE>(job, t, local, gbase);
    const int64_t nch = crun_chunks(s.n, s.w);
    const int64_t c0 = local * job.run;
    crun_body<T>(s, c0, min(nch, c0 + job.run), sm);
  }
}

// ================================================================ batched
// Descriptors and per-path tile prefix sums for a batch of S series (the
// path of a series -- tile kernel of lag 1..4, or chunk kernel -- comes
// from the plan's strategy for its size class, batch_path), three passes:
//  1. k_batched_count (G <= 1024 workgroups, contiguous ranges of `per`
//     series, a multiple of 256): descriptors, each series' tile count on
//     every path (zero but on its own), written in place, and the
//     workgroup's totals per path;
//  2. k_batched_scan (one workgroup): exclusive scan of the G totals of
//     every path;
//  3. k_batched_fix (G workgroups): each range's exclusive scans plus their
//     offsets, in place; entry S of each path gets its total.
// (A single-workgroup scan over the series took 0.42 ms for 100,000.)
// Layout of pre: path p's prefix array at pre + p (S + 1); the totals at
// part = pre + kBatchNP (S + 1): part[p G + g], grand totals part[kBatchNP G + p].

template <class T>
__global__ __launch_bounds__(256) void k_batched_count(const T* d_in, const int64_t* in_off, const int64_t* wins,
                                                       const int64_t* out_off, int64_t S, T* d_max, T* d_min,
                                                       Series<T>* descs, int64_t* pre, BatchPlan plan, int64_t per) {
  constexpr int NP = kBatchNP;
  __shared__ int64_t red[NP][4];
  const int64_t k0 = (int64_t)blockIdx.x * per;
  const int64_t run = (int64_t)plan.run_subtiles * kTileOut;
  int64_t tot[NP];
#pragma unroll
  for (int q = 0; q < NP; ++q) tot[q] = 0;
  for (int64_t j = 0; j < per / 256; ++j) {
    const int64_t k = k0 + j * 256 + threadIdx.x;
    if (k >= S) break;
    const int64_t n = in_off[k + 1] - in_off[k], w = wins[k];
    Series<T> d;
    d.a = d_in + in_off[k];
    d.b = nullptr;
    d.na = n;
    d.n = n;
    d.w = w;
    d.omax = d_max ? d_max + out_off[k] : nullptr;
    d.omin = d_min ? d_min + out_off[k] : nullptr;
    d.carry = nullptr;
    descs[k] = d;
    const int path = batch_path(plan, n, w);
    const int64_t c = batch_tiles(path, n, w, run);
#pragma unroll
    for (int q = 0; q < NP; ++q) {
      const int64_t v = q == path ? c : 0;
      pre[q * (S + 1) + k] = v;
      tot[q] += v;
    }
  }
  // workgroup totals
#pragma unroll
  for (int q = 0; q < NP; ++q) {
    for (int d = 32; d >= 1; d >>= 1) tot[q] += __shfl_xor(tot[q], d, 64);
    if ((threadIdx.x & 63) == 0) red[q][threadIdx.x >> 6] = tot[q];
  }
  __syncthreads();
  if (threadIdx.x < NP) {
    const int q = threadIdx.x;
    int64_t* part = pre + NP * (S + 1);
    part[(int64_t)q * gridDim.x + blockIdx.x] = red[q][0] + red[q][1] + red[q][2] + red[q][3];
  }
}

// Exclusive scan of the G (<= 1024) workgroup totals of every path, in
// place; part[kBatchNP G + p] gets path p's grand total.
__global__ __launch_bounds__(1024) void k_batched_scan(int G, int64_t* part) {
  constexpr int NP = kBatchNP;
  __shared__ int64_t sc[NP][1024];
  const int tid = threadIdx.x;
  int64_t own[NP];
#pragma unroll
  for (int q = 0; q < NP; ++q) {
    own[q] = tid < G ? part[q * G + tid] : 0;
    sc[q][tid] = own[q];
  }
  __syncthreads();
  for (int d = 1; d < 1024; d <<= 1) {
    int64_t x[NP];
#pragma unroll
    for (int q = 0; q < NP; ++q) x[q] = tid >= d ? sc[q][tid - d] : 0;
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NP; ++q) sc[q][tid] += x[q];
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < NP; ++q) {
    if (tid < G) part[q * G + tid] = sc[q][tid] - own[q];
    if (tid == 1023) part[NP * G + q] = sc[q][1023];
  }
}

// Each workgroup's range: exclusive scans of its counts plus its offsets
// (per / 256 consecutive series per thread, read twice).
__global__ __launch_bounds__(256) void k_batched_fix(int64_t S, int G, int64_t per, int64_t* pre) {
  constexpr int NP = kBatchNP;
  __shared__ int64_t wt[NP][4];
  const int64_t* part = pre + NP * (S + 1);
  const int64_t PT = per / 256;
  const int64_t k0 = (int64_t)blockIdx.x * per + (int64_t)threadIdx.x * PT;
  const int64_t k1 = min(S, k0 + PT);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  int64_t acc[NP], inc[NP];
#pragma unroll
  for (int q = 0; q < NP; ++q) {
    acc[q] = 0;
    for (int64_t k = k0; k < k1; ++k) acc[q] += pre[q * (S + 1) + k];
    // inclusive scan of the thread totals over the wavefront
    inc[q] = acc[q];
    for (int d = 1; d < 64; d <<= 1) {
      const int64_t x = __shfl_up(inc[q], d, 64);
      if (lane >= d) inc[q] += x;
    }
    if (lane == 63) wt[q][wv] = inc[q];
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < NP; ++q) {
    int64_t b = part[q * G + blockIdx.x];
    for (int o = 0; o < wv; ++o) b += wt[q][o];
    int64_t r = b + inc[q] - acc[q];  // exclusive
    int64_t* a = pre + q * (S + 1);
    for (int64_t k = k0; k < k1; ++k) {
      const int64_t v = a[k];
      a[k] = r;
      r += v;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) a[S] = part[NP * G + q];
  }
}

// Autotuner input: a pseudo-random pattern (a hashed position, small
// integers of the element type).
template <class T> __global__ void k_tune_fill(T* a, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    uint32_t h = (uint32_t)i * 0x9E3779B1u;
    h ^= h >> 15;
    h *= 0x85EBCA77u;
    h ^= h >> 13;
    gstore(a + i, (T)(h & 0x3FFF));
  }
}

// Serving batches: pieces of host <-> device copies, one workgroup per
// piece at a time, 16-byte vectors when source, destination and size allow
// (else 4-, 2-byte or single bytes), four vectors per thread in flight so
// that the PCIe latency of host reads is covered.
__global__ __launch_bounds__(256) void k_copy_pieces(const CopyPiece* pieces, int64_t np) {
  for (int64_t q = blockIdx.x; q < np; q += gridDim.x) {
    const CopyPiece c = pieces[q];
    const uintptr_t al = (uintptr_t)c.src | (uintptr_t)c.dst | (uintptr_t)c.bytes;
    const int tid = threadIdx.x;
    if ((al & 15) == 0) {
      const u32x4* s = (const u32x4*)c.src;
      u32x4* d = (u32x4*)c.dst;
      const int64_t nv = c.bytes / 16;
      for (int64_t i = tid; i < nv; i += 4 * 256) {
        u32x4 v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u)
          if (i + u * 256 < nv) v[u] = gload(s + i + u * 256);
#pragma unroll
        for (int u = 0; u < 4; ++u)
          if (i + u * 256 < nv) gstore(d + i + u * 256, v[u]);
      }
    } else if ((al & 3) == 0) {
      const uint32_t* s = (const uint32_t*)c.src;
      uint32_t* d = (uint32_t*)c.dst;
      for (int64_t i = tid; i < c.bytes / 4; i += 256) gstore(d + i, gload(s + i));
    } else if ((al & 1) == 0) {
      const uint16_t* s = (const uint16_t*)c.src;
      uint16_t* d = (uint16_t*)c.dst;
      for (int64_t i = tid; i < c.bytes / 2; i += 256) gstore(d + i, gload(s + i));
    } else {
      for (int64_t i = tid; i < c.bytes; i += 256) c.dst[i] = c.src[i];
    }
  }
}

// A push that completes no window: the new carry is simply the last
// min(n, w-1) samples of (carry ++ chunk).
template <class T> __global__ void k_carry_only(Series<T> s) {
  const int64_t keep = min(s.n, s.w - 1);
  const int64_t cs = s.n - keep;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < keep; i += (int64_t)gridDim.x * blockDim.x)
    gstore(s.carry + i, src_at(s, cs + i));
}

// ================================================================ launchers
template <class F> static hipError_t dispatch(int dtype, F&& f) {
  switch (dtype) {
    case 0: return f((float*)nullptr);
    case 1: return f((double*)nullptr);
    case 2: return f((int32_t*)nullptr);
    case 3: return f((uint16_t*)nullptr);
    default: return hipErrorInvalidValue;
  }
}

size_t series_bytes() { return sizeof(Series<float>); }  // pointer/int64 fields: same for every T

template <class T> static Series<T> make_series(const JobArgs& a) {
  Series<T> s;
  s.a = (const T*)a.a;
  s.b = (const T*)a.b;
  s.na = a.na;
  s.n = a.n;
  s.w = a.w;
  s.omax = (T*)a.omax;
  s.omin = (T*)a.omin;
  s.carry = (T*)a.carry;
  return s;
}

template <class T> static Job<T> make_job(const JobArgs& a) {
  Job<T> j;
  j.mode = a.mode;
  j.one = make_series<T>(a);
  j.ntiles = a.ntiles;
  j.descs = (const Series<T>*)a.descs;
  j.pre = a.pre;
  j.S = a.S;
  j.in = (const T*)a.in;
  j.ld_in = a.ld_in;
  j.n = a.n;
  j.w = a.w;
  j.omax = (T*)a.omax;
  j.omin = (T*)a.omin;
  j.ld_out = a.ld_out;
  j.tpr = a.tpr;
  j.run = a.run;
  j.amax = a.amax;
  j.amin = a.amin;
  j.ranges = a.ranges;
  j.ring.f = a.ring;
  j.ring.lg = a.ring_lg;
  j.ctl = a.ctl;
  return j;
}

static int cu_count() {
  static int cus = 0;
  if (!cus) {
    int dev = 0;
    hipGetDevice(&dev);
    hipDeviceProp_t p;
    if (hipGetDeviceProperties(&p, dev) == hipSuccess) cus = p.multiProcessorCount;
    if (cus <= 0) cus = 256;
  }
  return cus;
}

template <class K> static int occupancy_grid(K kernel, int threads) {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kernel, threads, 0) != hipSuccess || nb < 1) nb = 1;
  return nb * cu_count();
}

int grid_cap(int dtype, int strategy) {
  static int cap[8][4] = {};
  if (dtype < 0 || dtype > 3 || strategy < kStratTile || strategy > kStratTile4) return 0;
  int& c = cap[strategy - 1][dtype];
  if (!c) {
    (void)dispatch(dtype, [&](auto* p) {
      using T = std::remove_pointer_t<decltype(p)>;
      c = strategy == kStratTile    ? occupancy_grid(k_tile<kJobDescs, T>, kTileThreads)
          : strategy == kStratChunk ? occupancy_grid(k_chunk<kJobDescs, T>, kChunkThreads)
          : strategy == kStratArg   ? occupancy_grid(k_tile<kJobOne, T, true>, kTileThreads)
          : strategy == kStratTile2 ? occupancy_grid(k_tile<kJobOne, T, false, 2>, kTileThreads)
          : strategy == kStratArg2  ? occupancy_grid(k_tile<kJobOne, T, true, 2>, kTileThreads)
          : strategy == kStratTile3 ? occupancy_grid(k_tile<kJobOne, T, false, 3>, kTileThreads)
          : strategy == kStratTile4 ? occupancy_grid(k_tile<kJobOne, T, false, 4>, kTileThreads)
                                    : occupancy_grid(k_crun<kJobDescs, T>, kChunkThreads);
      return hipSuccess;
    });
  }
  return c;
}

template <class T, int V>
static hipError_t launch_long_v(const Series<T>& s, int64_t nch, int64_t K, T* ax, T* an, hipStream_t st) {
  const int g1 = (int)std::min<int64_t>(nch, (int64_t)cu_count() * 8);
  hipLaunchKernelGGL((k_chunk_agg<T, V>), dim3(g1), dim3(kChunkThreads), 0, st, s, ax, an);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  // whole columns per workgroup group: a multiple of K workgroups (no
  // workgroup waits on another, so the grid may exceed residency)
  const int64_t cap = occupancy_grid(k_chunk_col<T, V>, kChunkThreads);
  const int64_t g2 = std::max<int64_t>(1, cap / K) * K;
  if (g2 > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_chunk_col<T, V>), dim3((unsigned)g2), dim3(kChunkThreads), 0, st, s, (const T*)ax,
                     (const T*)an);
  return hipGetLastError();
}

template <class T, int V>
static hipError_t launch_long1_v(Series<T> s, int64_t K, uint64_t* rec, Ctl* ctl, hipStream_t st) {
  // outputs a step behind the records from K = 32 chunks per block on
  // (MAXMIN_LONG_DEFER=0 / =1 forces either: experiments, tests)
  const char* ed = getenv("MAXMIN_LONG_DEFER");
  const bool defer = ed ? ed[0] != '0' : K >= 32;
  auto* kern = defer ? &k_chunk_col1<T, V, true> : &k_chunk_col1<T, V, false>;
  // every workgroup resident: a multiple of K no larger than the device holds
  const int64_t cap = occupancy_grid(kern, kChunkThreads);
  const int64_t g = cap / K * K;
  if (g < K) return hipErrorNotSupported;  // fewer slots than one column group
  void* args[] = {(void*)&s, (void*)&rec, (void*)&ctl};
  return hipLaunchCooperativeKernel(reinterpret_cast<const void*>(kern), dim3((unsigned)g), dim3(kChunkThreads),
                                    args, 0, st);
}

static size_t elem_size(int dtype) { return dtype == 1 ? 8 : (dtype == 3 ? 2 : 4); }

int64_t long1_records(int dtype, int64_t n, int64_t w) {
  const int64_t cmax = int64_t(kChunkThreads) * long1_col_v(w, elem_size(dtype));
  const int64_t K = (w + cmax - 1) / cmax;
  return ((n + w - 1) / w) * K;
}

hipError_t launch_long1(int dtype, const JobArgs& a, uint64_t* rec, Ctl* ctl, hipStream_t st) {
  const int V = long1_col_v(a.w, elem_size(dtype));
  const int64_t cmax = int64_t(kChunkThreads) * V;
  const int64_t K = (a.w + cmax - 1) / cmax;
  if (chunk_count(a.n, a.w, cmax) <= 0) return hipSuccess;
  if (K < 2 || a.mode != kJobOne) return hipErrorInvalidValue;
  return dispatch(dtype, [&](auto* p) {
    using T = std::remove_pointer_t<decltype(p)>;
    const Series<T> s = make_series<T>(a);
    return V == kColVShort ? launch_long1_v<T, kColVShort>(s, K, rec, ctl, st)
                           : launch_long1_v<T, kChunkV>(s, K, rec, ctl, st);
  });
}

hipError_t launch_long(int dtype, const JobArgs& a, void* agg, hipStream_t st) {
  const int64_t cmax = long_chunk_max(a.w);
  const int64_t K = (a.w + cmax - 1) / cmax;
  const int64_t nch = chunk_count(a.n, a.w, cmax);
  if (nch <= 0) return hipSuccess;
  if (K < 2 || a.mode != kJobOne) return hipErrorInvalidValue;
  return dispatch(dtype, [&](auto* p) {
    using T = std::remove_pointer_t<decltype(p)>;
    const Series<T> s = make_series<T>(a);
    T* ax = (T*)agg;
    T* an = ax + nch;
    return long_col_v(a.w) == kColVShort ? launch_long_v<T, kColVShort>(s, nch, K, ax, an, st)
                                         : launch_long_v<T, kChunkV>(s, nch, K, ax, an, st);
  });
}

hipError_t launch_1d(int dtype, int strategy, const JobArgs& a, int grid, hipStream_t st) {
  return dispatch(dtype, [&](auto* p) {
    using T = std::remove_pointer_t<decltype(p)>;
    const Job<T> j = make_job<T>(a);
    const dim3 g(grid);
    if (strategy == kStratArg || strategy == kStratArg2) {
      if (a.mode != kJobOne || a.amax == nullptr || a.amin == nullptr) return hipErrorInvalidValue;
      if (strategy == kStratArg) {
        if (a.w > kTileMaxW) return hipErrorInvalidValue;
        hipLaunchKernelGGL((k_tile<kJobOne, T, true>), g, dim3(kTileThreads), 0, st, j);
      } else {
        if (a.w <= kTileMaxW || a.w > kTileMaxW2) return hipErrorInvalidValue;
        hipLaunchKernelGGL((k_tile<kJobOne, T, true, 2>), g, dim3(kTileThreads), 0, st, j);
      }
    } else if (strategy == kStratTile3 || strategy == kStratTile4) {
      // windows ending three or four sub-tiles after they start
      // (described series: the setup sends only such windows here)
      const int L = strategy == kStratTile3 ? 3 : 4;
      if (a.mode != kJobDescs && (a.w <= (L - 1) * (int64_t)kTileOut || a.w > L * (int64_t)kTileOut))
        return hipErrorInvalidValue;
      if (a.mode == kJobOne) {
        if (L == 3) hipLaunchKernelGGL((k_tile<kJobOne, T, false, 3>), g, dim3(kTileThreads), 0, st, j);
        else hipLaunchKernelGGL((k_tile<kJobOne, T, false, 4>), g, dim3(kTileThreads), 0, st, j);
      } else if (a.mode == kJobRows) {
        if (L == 3) hipLaunchKernelGGL((k_tile<kJobRows, T, false, 3>), g, dim3(kTileThreads), 0, st, j);
        else hipLaunchKernelGGL((k_tile<kJobRows, T, false, 4>), g, dim3(kTileThreads), 0, st, j);
      } else {
        if (L == 3) hipLaunchKernelGGL((k_tile<kJobDescs, T, false, 3>), g, dim3(kTileThreads), 0, st, j);
        else hipLaunchKernelGGL((k_tile<kJobDescs, T, false, 4>), g, dim3(kTileThreads), 0, st, j);
      }
    } else if (strategy == kStratTile2) {
      // the two-sub-tile emission lag needs every window to end past its
      // own sub-tile and at most two sub-tiles on
      if (a.mode != kJobDescs && (a.w <= kTileMaxW || a.w > kTileMaxW2)) return hipErrorInvalidValue;
      if (a.mode == kJobOne) hipLaunchKernelGGL((k_tile<kJobOne, T, false, 2>), g, dim3(kTileThreads), 0, st, j);
      else if (a.mode == kJobRows) hipLaunchKernelGGL((k_tile<kJobRows, T, false, 2>), g, dim3(kTileThreads), 0, st, j);
      else hipLaunchKernelGGL((k_tile<kJobDescs, T, false, 2>), g, dim3(kTileThreads), 0, st, j);
    } else if (strategy == kStratTile) {
      if (a.mode != kJobDescs && a.w > kTileMaxW) return hipErrorInvalidValue;
      if (a.mode == kJobOne) hipLaunchKernelGGL((k_tile<kJobOne, T>), g, dim3(kTileThreads), 0, st, j);
      else if (a.mode == kJobDescs) hipLaunchKernelGGL((k_tile<kJobDescs, T>), g, dim3(kTileThreads), 0, st, j);
      else hipLaunchKernelGGL((k_tile<kJobRows, T>), g, dim3(kTileThreads), 0, st, j);
    } else if (strategy == kStratRun) {
      if (a.mode == kJobOne) hipLaunchKernelGGL((k_crun<kJobOne, T>), g, dim3(kChunkThreads), 0, st, j);
      else if (a.mode == kJobDescs) hipLaunchKernelGGL((k_crun<kJobDescs, T>), g, dim3(kChunkThreads), 0, st, j);
      else hipLaunchKernelGGL((k_crun<kJobRows, T>), g, dim3(kChunkThreads), 0, st, j);
    } else {
      if (a.mode == kJobOne) hipLaunchKernelGGL((k_chunk<kJobOne, T>), g, dim3(kChunkThreads), 0, st, j);
      else if (a.mode == kJobDescs) hipLaunchKernelGGL((k_chunk<kJobDescs, T>), g, dim3(kChunkThreads), 0, st, j);
      else hipLaunchKernelGGL((k_chunk<kJobRows, T>), g, dim3(kChunkThreads), 0, st, j);
    }
    return hipGetLastError();
  });
}

hipError_t launch_copy_pieces(const CopyPiece* pieces, int64_t np, hipStream_t st) {
  if (np <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_copy_pieces, dim3((unsigned)std::min<int64_t>(np, 2048)), dim3(256), 0, st, pieces, np);
  return hipGetLastError();
}

hipError_t launch_tune_fill(int dtype, void* a, int64_t n, hipStream_t st) {
  return dispatch(dtype, [&](auto* p) {
    using T = std::remove_pointer_t<decltype(p)>;
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_tune_fill<T>, dim3((unsigned)std::min<int64_t>((n + 255) / 256, 8192)), dim3(256), 0, st,
                       (T*)a, n);
    return hipGetLastError();
  });
}

hipError_t launch_batched_setup(int dtype, const void* d_in, const int64_t* in_off, const int64_t* wins,
                                const int64_t* out_off, int64_t S, void* d_max, void* d_min, void* descs,
                                int64_t* pre, const BatchPlan& plan, hipStream_t st) {
  return dispatch(dtype, [&](auto* p) {
    using T = std::remove_pointer_t<decltype(p)>;
    if (S <= 0) return hipSuccess;
    if (plan.run_subtiles < 1) return hipErrorInvalidValue;
    // series per workgroup: a multiple of 256, at least 1024, at most
    // kBatchMaxGroups workgroups
    int64_t per = (S + kBatchMaxGroups - 1) / kBatchMaxGroups;
    per = std::max<int64_t>(1024, (per + 255) / 256 * 256);
    const int64_t G = (S + per - 1) / per;
    hipLaunchKernelGGL(k_batched_count<T>, dim3((unsigned)G), dim3(256), 0, st, (const T*)d_in, in_off, wins,
                       out_off, S, (T*)d_max, (T*)d_min, (Series<T>*)descs, pre, plan, per);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_batched_scan, dim3(1), dim3(1024), 0, st, (int)G, pre + kBatchNP * (S + 1));
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_batched_fix, dim3((unsigned)G), dim3(256), 0, st, S, (int)G, per, pre);
    return hipGetLastError();
  });
}

hipError_t launch_arg_combine(int dtype, const void* vx, const void* vn, const int64_t* ix, const int64_t* in_,
                              int64_t q, int64_t p, int F, int64_t nout, void* ox, void* on, int64_t* jx, int64_t* jn,
                              hipStream_t st) {
  if (nout <= 0) return hipSuccess;
  const int grid = (int)std::min<int64_t>((nout + 255) / 256, (int64_t)cu_count() * 16);
  return dispatch(dtype, [&](auto* ptr) {
    using T = std::remove_pointer_t<decltype(ptr)>;
    hipLaunchKernelGGL(k_argcombine<T>, dim3(grid), dim3(256), 0, st, (const T*)vx, (const T*)vn, ix, in_, q, p, F,
                       nout, (T*)ox, (T*)on, jx, jn);
    return hipGetLastError();
  });
}

hipError_t launch_env_ends(int dtype, const void* a, int64_t n, int64_t r, void* up, void* lo, hipStream_t st) {
  if (n <= 0 || r <= 0) return hipSuccess;
  return dispatch(dtype, [&](auto* p) {
    using T = std::remove_pointer_t<decltype(p)>;
    hipLaunchKernelGGL(k_env_ends<T>, dim3(2), dim3(256), 0, st, (const T*)a, n, r, (T*)up, (T*)lo);
    return hipGetLastError();
  });
}

hipError_t launch_env_batched(int dtype, const void* in, const int64_t* off, const int64_t* radii, int64_t S,
                              int64_t* wins, int64_t* oo, bool setup, void* up, void* lo, hipStream_t st) {
  if (S <= 0) return hipSuccess;
  if (setup) {
    const int g = (int)std::min<int64_t>((S + 256) / 256, 1024);
    hipLaunchKernelGGL(k_env_setup, dim3(g), dim3(256), 0, st, off, radii, S, wins, oo);
    return hipGetLastError();
  }
  const int g = (int)std::min<int64_t>((2 * S + 3) / 4, (int64_t)cu_count() * 32);
  hipError_t e = dispatch(dtype, [&](auto* p) {
    using T = std::remove_pointer_t<decltype(p)>;
    hipLaunchKernelGGL(k_env_ends_batched<T>, dim3(g), dim3(256), 0, st, (const T*)in, off, radii, S, (T*)up,
                       (T*)lo);
    return hipGetLastError();
  });
  if (e != hipSuccess) return e;
  return launch_env_short(dtype, in, off, radii, S, up, lo, st);
}

hipError_t launch_carry_only(int dtype, const JobArgs& a, hipStream_t st) {
  return dispatch(dtype, [&](auto* p) {
    using T = std::remove_pointer_t<decltype(p)>;
    hipLaunchKernelGGL(k_carry_only<T>, dim3(8), dim3(256), 0, st, make_series<T>(a));
    return hipGetLastError();
  });
}

}  // namespace mm
