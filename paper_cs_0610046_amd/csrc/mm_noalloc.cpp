// maxmin_filter_noalloc: maxmin_filter without any allocation, for callers
// that cannot allocate device memory (code under HIP graph capture, tight
// serving loops, harnesses that forbid hipMalloc).  Its only scratch memory
// is the file-scope array below.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>

#include "maxmin.h"
#include "mm_launch.hpp"

namespace {

// The long-window kernels' chunk aggregates (a max and a min per chunk).
// Each GPU the library runs on holds one copy until the process ends.
constexpr size_t kScratchBytes = size_t(32) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_scratch[kMaxDevices] = {};  // device address of `scratch` per device

// Device address of this device's copy of `scratch`, looked up once per
// device with that device current.  In host code the array's name is only a
// stand-in: kernels get this address.
int scratch_ptr(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return mm::set_error(MAXMIN_EDEVICE, "maxmin_filter_noalloc: hipGetDevice failed");
  if (dev < 0 || dev >= kMaxDevices) return mm::set_error(MAXMIN_EUNSUPPORTED, "maxmin_filter_noalloc: device id");
  std::lock_guard<std::mutex> g(g_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return mm::set_error(MAXMIN_EDEVICE, "maxmin_filter_noalloc: hipGetSymbolAddress(scratch) failed");
    g_scratch[dev] = p;
  }
  *out = g_scratch[dev];
  return MAXMIN_OK;
}

size_t esize(int dt) { return dt == MAXMIN_F64 ? 8 : (dt == MAXMIN_U16 ? 2 : (dt >= 0 && dt <= 3 ? 4 : 0)); }

}  // namespace

extern "C" int maxmin_filter_noalloc(int dtype, const void* d_in, int64_t n, int64_t w, void* d_max, void* d_min,
                                     void* stream) {
  const size_t s = esize(dtype);
  if (!s) return mm::set_error(MAXMIN_EINVAL, "maxmin_filter_noalloc: unknown dtype");
  if (w < 1) return mm::set_error(MAXMIN_EINVAL, "maxmin_filter_noalloc: window w < 1");
  if (n < 0) return mm::set_error(MAXMIN_EINVAL, "maxmin_filter_noalloc: n < 0");
  if (n < w) return mm::set_error(MAXMIN_OK, "");  // no complete window
  if (!d_in || (!d_max && !d_min)) return mm::set_error(MAXMIN_EINVAL, "maxmin_filter_noalloc: null pointer");
  if ((uintptr_t)d_in % s || (uintptr_t)d_max % s || (uintptr_t)d_min % s)
    return mm::set_error(MAXMIN_EINVAL, "maxmin_filter_noalloc: pointer not aligned to the element size");
  hipStream_t st = (hipStream_t)stream;
  mm::JobArgs a;
  a.mode = 0;
  a.a = d_in;
  a.na = n;
  a.n = n;
  a.w = w;
  a.omax = d_max;
  a.omin = d_min;
  hipError_t e;
  if (w <= mm::kTileMaxW4) {
    e = mm::launch_tile_series(dtype, a, st);  // no scratch
  } else {
    // chunk aggregates, then columns of chunks: pass 1 writes every
    // aggregate pass 2 reads, so nothing in the scratch needs clearing
    const int64_t nch = mm::chunk_count(n, w, mm::long_chunk_max(w));
    if ((uint64_t)nch > kScratchBytes / (2 * s))
      return mm::set_error(MAXMIN_EUNSUPPORTED,
                           "maxmin_filter_noalloc: the series needs more than the 32 MiB of scratch "
                           "(2 * chunks * element size) for this window");
    void* p = nullptr;
    const int r = scratch_ptr(&p);
    if (r) return r;
    e = mm::launch_long(dtype, a, p, st);
  }
  if (e != hipSuccess) return mm::set_error(MAXMIN_EDEVICE, "maxmin_filter_noalloc: kernel launch failed");
  return mm::set_error(MAXMIN_OK, "");
}
