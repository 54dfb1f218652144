// CPU oracle for the running max-min filter -- TEST INFRASTRUCTURE ONLY.
//
// Only the test suite, the smoke check and the benchmark's CPU-baseline leg
// load this library.  It shares no source, header, table or helper with the
// GPU library, and the GPU library never calls it.
//
// Paper: D. Lemire, "Streaming Maximum-Minimum Filter Using No More than Three
// Comparisons per Element".
//
// What is here:
//   * naive_*      the definition of the filter written out (Section 1: the
//                  max and min of a_i over every window [j, j+w)); the naive
//                  row of Table 1.
//   * Wedge<T>     the paper's streaming algorithm (Section 4, Algorithm 1):
//                  a monotonic wedge (lists U and L) updated one sample at a
//                  time, with zero stream latency (Section 1 definition).
//   * filter2d_*   the 2-D use of the 1-D filter: rows first, then columns
//                  (Section 1, image-processing paragraph).
//   * naive2d_*    the 2-D definition written out (max/min over every
//                  w_rows x w_cols rectangle), to pin filter2d.
//   * argnaive     the locations of the window maxima and minima, from the
//                  definition: the leftmost location attaining the window's
//                  max (min).  The paper notes that an implementation that
//                  stores locations gives this arg max/min filter at no
//                  extra cost (Section 5); it fixes no rule for ties.
//   * vhgw1, gk1, minmax3  other exact filters the paper reviews (van Herk /
//                  Gil-Werman, Gil-Kimmel, and the two-comparison w = 3
//                  algorithm), as cross-checks with comparison counts.
//   * envelope     the centered envelope (windows [i-r, i+r] truncated at
//                  the series ends), from the definition.
//   * argdeque     the same locations from a monotonic deque of locations
//                  that drops only strictly dominated entries (so equal
//                  values stay and the front is the leftmost), pinned to
//                  argnaive; linear time, for large tests.
//
// Every value operation is a comparison followed by a selection, so all
// results are exact for every dtype.  Indices are 64-bit (Section 5 advises
// 64-bit locations when processing streams).
//
// Readings of the paper taken here (ambiguous or garbled passages):
//   R1  0-based output index: out[j] covers [j, j+w) (the paper's pseudocode
//       is 1-based).
//   R2  valid mode only: n_out = max(0, n-w+1); w > n yields no output.
//   R3  Algorithm 1's inner while-loops test an element of U (or L) right
//       after an unconditional pop; we add the missing "list not empty"
//       guard.
//   R4  Algorithm 1 emits the window [i-w, i) at the top of iteration i, so
//       the last window is never emitted; emitting at the end of each
//       iteration (zero latency) emits every window, including the last.
//   R5  Algorithm 1 states w > 2; the wedge update is valid for every w >= 1
//       (w = 1 is the identity).
//   R6  Only comparisons between values are counted (Section 1 cost model);
//       emptiness and index tests are not.
//   R7  Locations: the paper's update sends an element equal to its
//       predecessor to L and so does not always return the leftmost minimum
//       among ties; the location outputs here follow one rule for both: the
//       leftmost location of the window's max (min).
#include <cstdint>
#include <cstring>
#include <deque>
#include <utility>
#include <vector>

namespace {

template <class T>
struct Wedge {
  // One entry of U or L: a location and the value stored there.  A stream
  // cannot keep a[] around, so the value travels with its location.
  typedef std::pair<int64_t, T> Entry;

  int64_t w;
  int64_t t;          // samples pushed so far; the next sample has index t
  T prev;             // a_{t-1}
  std::deque<Entry> U;  // locations of the running maxima (front = argmax)
  std::deque<Entry> L;  // locations of the running minima (front = argmin)
  int64_t ncmp;       // value comparisons made so far
  int64_t peak;       // largest size(U)+size(L) seen after an update

  explicit Wedge(int64_t w_) : w(w_), t(0), prev(), ncmp(0), peak(0) {}

  // Push one sample; returns true when the window ending at this sample is
  // complete, with its maximum and minimum in *mx / *mn.
  template <bool COUNT>
  bool push(T x, T* mx, T* mn) {
    if (t == 0) {
      // First sample: the wedge of a single point holds it in both lists.
      U.push_back(Entry(0, x));
      L.push_back(Entry(0, x));
    } else {
      // Compare the new sample with the previous one (the one comparison
      // every element pays).  t-1 is the last location of both U and L.
      if (COUNT) ++ncmp;
      if (x > prev) {
        // The new value beats a_{t-1}: a_{t-1} cannot be a future maximum,
        // so it leaves U (it stays in L); then drop every remaining
        // maximum candidate that x beats.
        U.pop_back();
        while (!U.empty()) {  // R3
          if (COUNT) ++ncmp;
          if (x > U.back().second) U.pop_back();
          else break;
        }
      } else {
        // Symmetric case on the minimum side: a_{t-1} leaves L, then every
        // minimum candidate larger than x goes.
        L.pop_back();
        while (!L.empty()) {  // R3
          if (COUNT) ++ncmp;
          if (x < L.back().second) L.pop_back();
          else break;
        }
      }
      // Append the new location to both lists.
      U.push_back(Entry(t, x));
      L.push_back(Entry(t, x));
      // Location t-w just left the window: it sits in at most one list, at
      // its front.
      if (U.front().first == t - w) U.pop_front();
      else if (L.front().first == t - w) L.pop_front();
    }
    prev = x;
    ++t;
    int64_t sz = (int64_t)U.size() + (int64_t)L.size();
    if (sz > peak) peak = sz;
    if (t >= w) {  // R4: zero-latency emission of window [t-w, t)
      *mx = U.front().second;
      *mn = L.front().second;
      return true;
    }
    return false;
  }

  // Push m samples, writing the windows they complete; returns how many.
  template <bool COUNT>
  int64_t push_many(const T* a, int64_t m, T* mx, T* mn) {
    int64_t k = 0;
    for (int64_t i = 0; i < m; ++i) {
      T M, N;
      if (push<COUNT>(a[i], &M, &N)) {
        mx[k] = M;
        mn[k] = N;
        ++k;
      }
    }
    return k;
  }
};

// The definition: max and min over each window [j, j+w), by scanning it.
template <class T>
void naive(const T* a, int64_t n, int64_t w, T* mx, T* mn) {
  for (int64_t j = 0; j + w <= n; ++j) {
    T M = a[j], N = a[j];
    for (int64_t i = j + 1; i < j + w; ++i) {
      if (a[i] > M) M = a[i];
      if (a[i] < N) N = a[i];
    }
    mx[j] = M;
    mn[j] = N;
  }
}

template <class T>
int64_t wedge_filter(const T* a, int64_t n, int64_t w, T* mx, T* mn,
                     int64_t* ncmp, int64_t* peak) {
  Wedge<T> s(w);
  int64_t k;
  if (ncmp) k = s.template push_many<true>(a, n, mx, mn);
  else k = s.template push_many<false>(a, n, mx, mn);
  if (ncmp) *ncmp = s.ncmp;
  if (peak) *peak = s.peak;
  return k;
}

// 2-D filter: the 1-D filter on each row, then on each column of the
// row-filtered images (max of the max-image, min of the min-image).
template <class T>
void filter2d(const T* a, int64_t rows, int64_t cols, int64_t ld, int64_t wr,
              int64_t wc, T* mx, T* mn, int64_t ldo) {
  int64_t oc = cols - wc + 1, orows = rows - wr + 1;
  if (oc <= 0 || orows <= 0) return;
  std::vector<T> rmax((size_t)(rows * oc)), rmin((size_t)(rows * oc));
  for (int64_t r = 0; r < rows; ++r)
    wedge_filter<T>(a + r * ld, cols, wc, &rmax[(size_t)(r * oc)],
                    &rmin[(size_t)(r * oc)], nullptr, nullptr);
  std::vector<T> col((size_t)rows), o1((size_t)orows), o2((size_t)orows);
  for (int64_t c = 0; c < oc; ++c) {
    for (int64_t r = 0; r < rows; ++r) col[(size_t)r] = rmax[(size_t)(r * oc + c)];
    wedge_filter<T>(col.data(), rows, wr, o1.data(), o2.data(), nullptr, nullptr);
    for (int64_t r = 0; r < orows; ++r) mx[r * ldo + c] = o1[(size_t)r];
    for (int64_t r = 0; r < rows; ++r) col[(size_t)r] = rmin[(size_t)(r * oc + c)];
    wedge_filter<T>(col.data(), rows, wr, o1.data(), o2.data(), nullptr, nullptr);
    for (int64_t r = 0; r < orows; ++r) mn[r * ldo + c] = o2[(size_t)r];
  }
}

// 2-D definition: max/min over each wr x wc rectangle, scanned directly.
template <class T>
void naive2d(const T* a, int64_t rows, int64_t cols, int64_t ld, int64_t wr,
             int64_t wc, T* mx, T* mn, int64_t ldo) {
  for (int64_t r = 0; r + wr <= rows; ++r)
    for (int64_t c = 0; c + wc <= cols; ++c) {
      T M = a[r * ld + c], N = M;
      for (int64_t i = r; i < r + wr; ++i)
        for (int64_t k = c; k < c + wc; ++k) {
          T v = a[i * ld + k];
          if (v > M) M = v;
          if (v < N) N = v;
        }
      mx[r * ldo + c] = M;
      mn[r * ldo + c] = N;
    }
}

// Locations (0-based, in the series) of the leftmost max and min of every
// window, scanned directly.
template <class T>
void argnaive(const T* a, int64_t n, int64_t w, int64_t* amx, int64_t* amn) {
  for (int64_t j = 0; j + w <= n; ++j) {
    int64_t im = j, in = j;
    for (int64_t i = j + 1; i < j + w; ++i) {
      if (a[i] > a[im]) im = i;  // strict: an equal later value never wins
      if (a[i] < a[in]) in = i;
    }
    amx[j] = im;
    amn[j] = in;
  }
}

// Same result in linear time: U holds locations with non-increasing values
// (front = leftmost max of the window), L non-decreasing (front = leftmost
// min).  A new value removes only the entries it strictly dominates.
template <class T>
void argdeque(const T* a, int64_t n, int64_t w, int64_t* amx, int64_t* amn) {
  std::deque<int64_t> U, L;
  for (int64_t i = 0; i < n; ++i) {
    const T x = a[i];
    while (!U.empty() && a[U.back()] < x) U.pop_back();
    U.push_back(i);
    while (!L.empty() && a[L.back()] > x) L.pop_back();
    L.push_back(i);
    if (U.front() <= i - w) U.pop_front();
    if (L.front() <= i - w) L.pop_front();
    if (i >= w - 1) {
      amx[i - w + 1] = U.front();
      amn[i - w + 1] = L.front();
    }
  }
}

// Centered envelope of radius r: the max and min over
// [max(0, i-r), min(n-1, i+r)] for every i (windows truncated at the series
// ends), scanned directly.  The paper cites the use of a precomputed
// max-min filter to bound the time warping distance (Section 1).
template <class T>
void envelope(const T* a, int64_t n, int64_t r, T* up, T* lo) {
  for (int64_t i = 0; i < n; ++i) {
    const int64_t j0 = i - r < 0 ? 0 : i - r, j1 = i + r > n - 1 ? n - 1 : i + r;
    T M = a[j0], N = a[j0];
    for (int64_t j = j0 + 1; j <= j1; ++j) {
      if (a[j] > M) M = a[j];
      if (a[j] < N) N = a[j];
    }
    up[i] = M;
    lo[i] = N;
  }
}

// ------------------------------------------------ cross-check algorithms
// Other exact max-min filters the paper reviews (Related Work, and the
// proposition on w = 3 in the lower-bound section), written from their
// descriptions, with value comparisons counted.  They give the same outputs
// as the definition by a different route and check the paper's comparison
// bounds for them.

// One direction of a filter: better(x, y) is x > y (max) or x < y (min).
template <class T, bool MAX>
struct Better {
  int64_t* n;
  bool operator()(T x, T y) const {
    ++*n;
    return MAX ? x > y : x < y;
  }
};
// the better of x and y, x on ties
template <class T, class C> T pick(T x, T y, C& c) { return c(y, x) ? y : x; }

// van Herk / Gil-Werman: blocks of w; prefix extrema over each block
// (w-1 comparisons), suffix extrema over all but its first position (w-2);
// the window starting at a block start is that block (its last prefix), any
// other window is the suffix of its first block against the prefix of the
// next (1 comparison): 3w-4 per block and direction.
template <class T, bool MAX>
void vhgw1(const T* a, int64_t n, int64_t w, T* out, int64_t* cnt) {
  Better<T, MAX> c{cnt};
  std::vector<T> P((size_t)n), S((size_t)n);
  for (int64_t b0 = 0; b0 < n; b0 += w) {
    const int64_t b1 = b0 + w < n ? b0 + w : n;
    P[(size_t)b0] = a[b0];
    for (int64_t i = b0 + 1; i < b1; ++i) P[(size_t)i] = pick(P[(size_t)(i - 1)], a[i], c);
    S[(size_t)(b1 - 1)] = a[b1 - 1];
    for (int64_t i = b1 - 2; i > b0; --i) S[(size_t)i] = pick(S[(size_t)(i + 1)], a[i], c);
  }
  for (int64_t j = 0; j + w <= n; ++j)
    out[j] = j % w == 0 ? P[(size_t)(j + w - 1)] : pick(S[(size_t)j], P[(size_t)(j + w - 1)], c);
}

// Gil-Kimmel, both improvements: (1) a block's prefix extrema stop changing
// after its best element and its suffix extrema before it, so compute the
// prefix over the first half and the suffix over the second, compare their
// ends once to learn which half holds the best, and compute only the other
// two halves that can still change; (2) across the windows starting in a
// block, the suffix term only worsens and the prefix term only improves, so
// a binary search finds where the prefix takes over.
template <class T, bool MAX>
void gk1(const T* a, int64_t n, int64_t w, T* out, int64_t* cnt) {
  Better<T, MAX> c{cnt};
  std::vector<T> P((size_t)n), S((size_t)n);
  for (int64_t b0 = 0; b0 < n; b0 += w) {
    const int64_t b1 = b0 + w < n ? b0 + w : n, len = b1 - b0, q = (len + 1) / 2;
    P[(size_t)b0] = a[b0];
    for (int64_t i = b0 + 1; i < b0 + q; ++i) P[(size_t)i] = pick(P[(size_t)(i - 1)], a[i], c);
    S[(size_t)(b1 - 1)] = a[b1 - 1];
    for (int64_t i = b1 - 2; i >= b0 + q; --i) S[(size_t)i] = pick(S[(size_t)(i + 1)], a[i], c);
    if (q == len) continue;  // a one-element block
    const bool first = !c(S[(size_t)(b0 + q)], P[(size_t)(b0 + q - 1)]);  // ties: the first half
    if (first) {
      for (int64_t i = b0 + q; i < b1; ++i) P[(size_t)i] = P[(size_t)(b0 + q - 1)];
      for (int64_t i = b0 + q - 1; i > b0; --i) S[(size_t)i] = pick(S[(size_t)(i + 1)], a[i], c);
    } else {
      for (int64_t i = b0 + q; i < b1; ++i) P[(size_t)i] = pick(P[(size_t)(i - 1)], a[i], c);
      for (int64_t i = b0 + q - 1; i > b0; --i) S[(size_t)i] = S[(size_t)(b0 + q)];
    }
  }
  for (int64_t b0 = 0; b0 + w <= n; b0 += w) {
    out[b0] = P[(size_t)(b0 + w - 1)];  // the window is the block
    // windows j in (b0, e): the first j whose prefix term is at least as good
    const int64_t e = b0 + w < n - w + 1 ? b0 + w : n - w + 1;
    int64_t lo = b0 + 1, hi = e;  // answer in [lo, hi]; hi = e: never
    while (lo < hi) {
      const int64_t mid = lo + (hi - lo) / 2;
      if (!c(S[(size_t)mid], P[(size_t)(mid + w - 1)])) hi = mid;
      else lo = mid + 1;
    }
    for (int64_t j = b0 + 1; j < e; ++j) out[j] = j < lo ? S[(size_t)j] : P[(size_t)(j + w - 1)];
  }
}

template <class T>
void vhgw(const T* a, int64_t n, int64_t w, T* mx, T* mn, int64_t* cnt) {
  vhgw1<T, true>(a, n, w, mx, cnt);
  vhgw1<T, false>(a, n, w, mn, cnt);
}

template <class T>
void gil_kimmel(const T* a, int64_t n, int64_t w, T* mx, T* mn, int64_t* cnt) {
  gk1<T, true>(a, n, w, mx, cnt);
  gk1<T, false>(a, n, w, mn, cnt);
}

// w = 3 with two comparisons per element (the paper's proposition): the
// order of the last two samples is known from the previous step, so
// comparing the new sample with each of them orders all three.
template <class T>
void minmax3(const T* a, int64_t n, T* mx, T* mn, int64_t* cnt) {
  if (n < 3) return;
  ++*cnt;
  bool up = a[1] > a[0];  // a[i-1] > a[i-2]
  for (int64_t i = 2; i < n; ++i) {
    const bool c1 = a[i] > a[i - 1], c2 = a[i] > a[i - 2];
    *cnt += 2;
    const T hi2 = up ? a[i - 1] : a[i - 2], lo2 = up ? a[i - 2] : a[i - 1];
    mx[i - 2] = (up ? c1 : c2) ? a[i] : hi2;  // a[i] beats the larger of the two
    mn[i - 2] = (up ? c2 : c1) ? lo2 : a[i];  // a[i] above the smaller: that one
    up = c1;
  }
}

// dtype codes shared with the Python wrapper: 0 f32, 1 f64, 2 i32, 3 u16.
struct StreamBox {
  int dt;
  void* p;
};

}  // namespace

#define ORACLE_DISPATCH(dt, CALL)                 \
  switch (dt) {                                   \
    case 0: { typedef float T; CALL; break; }     \
    case 1: { typedef double T; CALL; break; }    \
    case 2: { typedef int32_t T; CALL; break; }   \
    case 3: { typedef uint16_t T; CALL; break; }  \
    default: return -1;                           \
  }

extern "C" {

int oracle_naive(int dt, const void* a, int64_t n, int64_t w, void* mx, void* mn) {
  if (w < 1 || n < 0) return -1;
  ORACLE_DISPATCH(dt, naive<T>((const T*)a, n, w, (T*)mx, (T*)mn));
  return 0;
}

// One-shot wedge filter.  ncmp / peak may be null (then nothing is counted).
int64_t oracle_wedge(int dt, const void* a, int64_t n, int64_t w, void* mx, void* mn,
                     int64_t* ncmp, int64_t* peak) {
  if (w < 1 || n < 0) return -1;
  int64_t k = 0;
  ORACLE_DISPATCH(dt, k = wedge_filter<T>((const T*)a, n, w, (T*)mx, (T*)mn, ncmp, peak));
  return k;
}

void* oracle_stream_create(int dt, int64_t w) {
  if (w < 1) return nullptr;
  StreamBox* b = new StreamBox;
  b->dt = dt;
  switch (dt) {
    case 0: b->p = new Wedge<float>(w); break;
    case 1: b->p = new Wedge<double>(w); break;
    case 2: b->p = new Wedge<int32_t>(w); break;
    case 3: b->p = new Wedge<uint16_t>(w); break;
    default: delete b; return nullptr;
  }
  return b;
}

// Push m samples; returns the number of completed windows written.
int64_t oracle_stream_push(void* h, const void* a, int64_t m, void* mx, void* mn) {
  StreamBox* b = (StreamBox*)h;
  int64_t k = 0;
  ORACLE_DISPATCH(b->dt, k = ((Wedge<T>*)b->p)->template push_many<true>((const T*)a, m, (T*)mx, (T*)mn));
  return k;
}

// Samples pushed, comparisons made, and the peak wedge size so far.
int oracle_stream_stats(void* h, int64_t* t, int64_t* ncmp, int64_t* peak) {
  StreamBox* b = (StreamBox*)h;
  ORACLE_DISPATCH(b->dt, {
    Wedge<T>* s = (Wedge<T>*)b->p;
    *t = s->t;
    *ncmp = s->ncmp;
    *peak = s->peak;
  });
  return 0;
}

void oracle_stream_destroy(void* h) {
  StreamBox* b = (StreamBox*)h;
  if (!b) return;
  switch (b->dt) {
    case 0: delete (Wedge<float>*)b->p; break;
    case 1: delete (Wedge<double>*)b->p; break;
    case 2: delete (Wedge<int32_t>*)b->p; break;
    case 3: delete (Wedge<uint16_t>*)b->p; break;
  }
  delete b;
}

int oracle_filter2d(int dt, const void* a, int64_t rows, int64_t cols, int64_t ld,
                    int64_t wr, int64_t wc, void* mx, void* mn, int64_t ldo) {
  if (wr < 1 || wc < 1 || rows < 0 || cols < 0 || ld < cols) return -1;
  ORACLE_DISPATCH(dt, filter2d<T>((const T*)a, rows, cols, ld, wr, wc, (T*)mx, (T*)mn, ldo));
  return 0;
}

int oracle_naive2d(int dt, const void* a, int64_t rows, int64_t cols, int64_t ld,
                   int64_t wr, int64_t wc, void* mx, void* mn, int64_t ldo) {
  if (wr < 1 || wc < 1 || rows < 0 || cols < 0 || ld < cols) return -1;
  ORACLE_DISPATCH(dt, naive2d<T>((const T*)a, rows, cols, ld, wr, wc, (T*)mx, (T*)mn, ldo));
  return 0;
}

int oracle_argnaive(int dt, const void* a, int64_t n, int64_t w, int64_t* amx, int64_t* amn) {
  if (w < 1 || n < 0) return -1;
  ORACLE_DISPATCH(dt, argnaive<T>((const T*)a, n, w, amx, amn));
  return 0;
}

int oracle_argdeque(int dt, const void* a, int64_t n, int64_t w, int64_t* amx, int64_t* amn) {
  if (w < 1 || n < 0) return -1;
  ORACLE_DISPATCH(dt, argdeque<T>((const T*)a, n, w, amx, amn));
  return 0;
}

int oracle_envelope(int dt, const void* a, int64_t n, int64_t r, void* up, void* lo) {
  if (r < 0 || n < 0) return -1;
  ORACLE_DISPATCH(dt, envelope<T>((const T*)a, n, r, (T*)up, (T*)lo));
  return 0;
}

int64_t oracle_vhgw(int dt, const void* a, int64_t n, int64_t w, void* mx, void* mn) {
  if (w < 1 || n < 0) return -1;
  int64_t k = 0;
  ORACLE_DISPATCH(dt, vhgw<T>((const T*)a, n, w, (T*)mx, (T*)mn, &k));
  return k;
}

int64_t oracle_gil_kimmel(int dt, const void* a, int64_t n, int64_t w, void* mx, void* mn) {
  if (w < 1 || n < 0) return -1;
  int64_t k = 0;
  ORACLE_DISPATCH(dt, gil_kimmel<T>((const T*)a, n, w, (T*)mx, (T*)mn, &k));
  return k;
}

int64_t oracle_minmax3(int dt, const void* a, int64_t n, void* mx, void* mn) {
  if (n < 0) return -1;
  int64_t k = 0;
  ORACLE_DISPATCH(dt, minmax3<T>((const T*)a, n, (T*)mx, (T*)mn, &k));
  return k;
}

}  // extern "C"
