// Serving engine: admission by an HBM budget, continuous batching over
// several HIP streams ("lanes"), device-resident stream carries, completion
// by events.  Host code only; every filter runs in the gfx950 kernels through
// the same batched launches as maxmin_filter_batched.
//
// Life of a request:
//   submit (any thread) -> pending FIFO, arrival time stamped
//   scheduler thread    -> admits requests in FIFO order while the arena
//                          (one hipMalloc of `budget` bytes, first-fit) has
//                          room; forms one batch per lane; per batch:
//                          H2D inputs, H2D descriptors, batched tile and
//                          chunk launches (one per dtype present), D2H
//                          outputs, event record
//   poller thread       -> sees the event, stamps completion, frees the
//                          batch's arena blocks, wakes the scheduler
//   poll (caller)       -> collects finished requests with their latency
// Requests that arrive while earlier batches are on the GPU go into the next
// batch as soon as memory frees up; batches on different lanes overlap on
// the device.  A stream's pushes always use the same lane (stream order)
// and at most one of them enters a batch (each reads the carry the previous
// one writes).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstdio>
#include <cstdlib>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <set>
#include <thread>
#include <vector>

#include "maxmin.h"
#include "mm_launch.hpp"

namespace {

using Clock = std::chrono::steady_clock;

size_t esize(int dt) { return dt == MAXMIN_F64 ? 8 : (dt == MAXMIN_U16 ? 2 : (dt >= 0 && dt <= 3 ? 4 : 0)); }

// First-fit allocator over one device block (offsets, 256-byte granules).
struct Arena {
  char* base = nullptr;
  int64_t size = 0;
  int64_t used = 0;
  std::map<int64_t, int64_t> free_;  // offset -> length
  static int64_t up(int64_t b) { return (b + 255) & ~int64_t(255); }
  int64_t alloc(int64_t bytes) {
    bytes = up(std::max<int64_t>(bytes, 1));
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        const int64_t off = it->first, rest = it->second - bytes;
        free_.erase(it);
        if (rest) free_[off + bytes] = rest;
        used += bytes;
        return off;
      }
    }
    return -1;
  }
  void release(int64_t off, int64_t bytes) {
    bytes = up(std::max<int64_t>(bytes, 1));
    used -= bytes;
    auto it = free_.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
};

enum { kFilter = 0, kPush = 1 };

struct Req {
  int64_t id = 0;
  int kind = kFilter;
  int dt = 0;
  int64_t n = 0;  // samples of this request (filter length or chunk size)
  int64_t w = 0;
  int64_t sid = 0;
  const void* h_in = nullptr;
  void* h_max = nullptr;
  void* h_min = nullptr;
  Clock::time_point t_arrive, t_done;
  int64_t nout = 0;
  int status = MAXMIN_OK;
  int64_t off = -1, bytes = 0;  // arena block: input, then max, then min outputs
  mm::Series<float> ser{};      // what the kernels see (pointer fields only: same layout for every dtype)
  bool carry_only = false;
  // device addresses of the host buffers when they are pinned and mapped
  // (the batch's copy kernels move them); null: hipMemcpyAsync per buffer
  const char* d_hin = nullptr;
  char* d_hmax = nullptr;
  char* d_hmin = nullptr;
};

// Device address of host memory the GPU can reach (pinned and mapped), or
// null for pageable memory.
const void* mapped(const void* h) {
  if (!h) return nullptr;
  hipPointerAttribute_t a;
  if (hipPointerGetAttributes(&a, h) != hipSuccess) {
    (void)hipGetLastError();  // pageable memory reports an error; clear it
    return nullptr;
  }
  if (a.type != hipMemoryTypeHost || !a.devicePointer) return nullptr;
  return a.devicePointer;
}

// Pieces of at most kCopyPieceMax bytes for one copy.
void add_pieces(std::vector<mm::CopyPiece>& v, const char* src, char* dst, int64_t bytes) {
  for (int64_t o = 0; o < bytes; o += mm::kCopyPieceMax)
    v.push_back(mm::CopyPiece{src + o, dst + o, std::min<int64_t>(mm::kCopyPieceMax, bytes - o)});
}

struct EStream {
  int dt = 0;
  int64_t w = 0;
  int64_t t = 0;     // samples admitted so far
  int64_t off = -1;  // arena block holding the two carry buffers
  int cur = 0;       // which carry holds the latest samples
  int lane = 0;
  int64_t queued = 0;  // pushes submitted but not yet completed
  bool broken = false;  // a push's kernels reported a device error: later pushes fail
};

// Host slots (pinned) that receive a lane's look-back error word after each
// batch that ran the chunk kernel.
constexpr int64_t kErrSlots = 4096;

struct Batch {
  int lane = 0;
  std::vector<Req*> reqs;
  std::vector<char> host;  // host image of the descriptors (kept until completion)
  hipEvent_t ev = nullptr;
  int64_t slot = -1;  // error-word slot, or -1 when no chunk kernel ran
};

struct Lane {
  hipStream_t st = nullptr;
  std::deque<Batch*> inflight;
  char* desc = nullptr;  // descriptor buffer: batches on one lane run in order, so one suffices
  size_t desc_cap = 0;
  mm::Ctl* ctl = nullptr;       // the lane stream's look-back control words
  uint32_t* h_err = nullptr;    // kErrSlots pinned words
  int64_t next_slot = 0;
};

}  // namespace

struct maxmin_engine {
  Arena arena;
  int64_t max_batch = 256;
  // Back-pressure: at most this many requests wait for admission; a submit
  // beyond it fails with MAXMIN_EBUSY (MAXMIN_ENGINE_MAX_PENDING).
  int64_t max_pending = 4096;
  // Host <-> device copies of pinned, mapped buffers below copy_max bytes by
  // the batch's copy kernels; larger ones (and pageable memory) by one
  // hipMemcpyAsync each.  On MI355X a copy engine spends ~10 us per copy
  // (64 KiB copies ran at 6 GB/s; one 1 GiB copy at 57 GB/s), while a kernel
  // moves many small buffers at once; a large buffer is better left to the
  // copy engines, which run beside the kernels.  MAXMIN_ENGINE_COPIES=memcpy
  // sends every buffer to the copy engines, MAXMIN_ENGINE_COPY_MAX sets the
  // size limit (experiments, tests).
  bool copy_kernels = true;
  int64_t copy_max = int64_t(1) << 20;
  std::vector<Lane> lanes;
  std::mutex mu;
  std::condition_variable cv_sched, cv_poll, cv_done;
  std::deque<Req*> pending;
  std::deque<Req*> done;
  std::map<int64_t, EStream> streams;
  std::thread sched, poller;
  bool stop = false;
  int64_t next_id = 1, next_sid = 1;
  int rr = 0;
  int device = 0;
  int64_t n_submitted = 0, n_done = 0, n_batches = 0, n_rejected = 0, elems_done = 0, peak_used = 0;
  int64_t n_busy = 0;  // submissions refused by back-pressure
  int64_t in_system = 0;  // submitted and not yet collected as done
  int64_t reserved = 0;   // budget held by open streams' carries
  // Fault injection for tests (MAXMIN_ENGINE_INJECT="launch:K" or "err:K"):
  // the K-th batch launched fails before enqueuing anything, or reports the
  // look-back error word as set.  0 = off.
  int64_t inject_launch = 0, inject_err = 0, launch_seq = 0;

  void scheduler_loop();
  void poller_loop();
  bool admit(Req* r, std::set<int64_t>& used_sids, std::vector<std::vector<Req*>>& per_lane);
  void launch(int lane, std::vector<Req*>& reqs);
  void finish(Req* r, int status);
};

namespace {

// Descriptor image for one dtype group of a batch: S series, then the tile
// and chunk prefix sums (S+1 int64 each).
struct Group {
  int dt;
  std::vector<Req*> reqs;
};

}  // namespace

void maxmin_engine::finish(Req* r, int status) {
  if (r->kind == kPush) {
    auto it = streams.find(r->sid);
    if (it != streams.end()) --it->second.queued;
  }
  r->status = status;
  r->t_done = Clock::now();
  done.push_back(r);
  ++n_done;
  cv_done.notify_all();
}

// Try to admit the head request (lock held).  Returns false when admission
// must stop for now (memory, or a second push of a stream in this batch).
bool maxmin_engine::admit(Req* r, std::set<int64_t>& used_sids, std::vector<std::vector<Req*>>& per_lane) {
  const int64_t s = (int64_t)esize(r->dt);
  if (r->kind == kFilter) {
    r->nout = std::max<int64_t>(0, r->n - r->w + 1);
    if (r->nout == 0) {  // no window: nothing to compute
      finish(r, MAXMIN_OK);
      return true;
    }
    r->bytes = Arena::up(r->n * s) + 2 * Arena::up(r->nout * s);
    if (r->bytes > arena.size - reserved) {  // could never fit: reject rather than wait forever
      ++n_rejected;
      finish(r, MAXMIN_ENOMEM);
      return true;
    }
    r->off = arena.alloc(r->bytes);
    if (r->off < 0) return false;
    char* p = arena.base + r->off;
    r->ser.a = (const float*)p;
    r->ser.b = (const float*)p;
    r->ser.na = r->n;
    r->ser.n = r->n;
    r->ser.w = r->w;
    r->ser.omax = (float*)(p + Arena::up(r->n * s));
    r->ser.omin = (float*)(p + Arena::up(r->n * s) + Arena::up(r->nout * s));
    r->ser.carry = nullptr;
    per_lane[rr++ % per_lane.size()].push_back(r);
    return true;
  }
  // stream push
  auto it = streams.find(r->sid);
  if (it == streams.end()) {
    finish(r, MAXMIN_EINVAL);
    return true;
  }
  if (used_sids.count(r->sid)) return false;
  EStream& es = it->second;
  if (es.broken) {
    finish(r, MAXMIN_EDEVICE);
    return true;
  }
  const int64_t c = std::min(es.t, es.w - 1);
  const int64_t total = c + r->n;
  r->nout = std::max<int64_t>(0, total - es.w + 1);
  r->bytes = Arena::up(r->n * s) + 2 * Arena::up(std::max<int64_t>(r->nout, 1) * s);
  if (r->bytes > arena.size - reserved) {
    ++n_rejected;
    finish(r, MAXMIN_ENOMEM);
    return true;
  }
  r->off = arena.alloc(r->bytes);
  if (r->off < 0) return false;
  char* p = arena.base + r->off;
  char* carry = arena.base + es.off;
  const int64_t cbytes = Arena::up(std::max<int64_t>(1, es.w - 1) * s);
  r->ser.a = (const float*)(carry + es.cur * cbytes);
  r->ser.na = c;
  r->ser.b = (const float*)p;
  r->ser.n = total;
  r->ser.w = es.w;
  r->ser.omax = (float*)(p + Arena::up(r->n * s));
  r->ser.omin = (float*)(p + Arena::up(r->n * s) + Arena::up(std::max<int64_t>(r->nout, 1) * s));
  r->ser.carry = es.w > 1 ? (float*)(carry + (1 - es.cur) * cbytes) : nullptr;
  r->carry_only = r->nout == 0;
  es.cur = 1 - es.cur;
  es.t += r->n;
  used_sids.insert(r->sid);
  per_lane[es.lane].push_back(r);
  return true;
}

void maxmin_engine::launch(int lane, std::vector<Req*>& reqs) {
  Lane& L = lanes[lane];
  for (;;) {  // every in-flight batch of the lane may hold an error-word slot
    {
      std::lock_guard<std::mutex> lk(mu);
      if ((int64_t)L.inflight.size() < kErrSlots) break;
    }
    std::this_thread::sleep_for(std::chrono::microseconds(50));
  }
  Batch* b = new Batch;
  b->lane = lane;
  b->reqs = reqs;
  const int64_t seq = ++launch_seq;
  hipError_t e = seq == inject_launch ? hipErrorLaunchFailure : hipSuccess;
  bool chunked = false;
  // inputs: pieces for the gather kernel (mapped host buffers), else copies
  std::vector<mm::CopyPiece> pin, pout;
  for (Req* r : reqs) {
    const size_t s = esize(r->dt);
    const void* dst = r->kind == kFilter ? (const void*)r->ser.a : (const void*)r->ser.b;
    if (r->n <= 0) continue;
    const int64_t bytes = r->n * (int64_t)s;
    if (r->d_hin && bytes <= copy_max) add_pieces(pin, r->d_hin, (char*)dst, bytes);
    else if (e == hipSuccess) e = hipMemcpyAsync((void*)dst, r->h_in, (size_t)bytes, hipMemcpyHostToDevice, L.st);
  }
  for (Req* r : reqs) {
    const int64_t bytes = r->nout * (int64_t)esize(r->dt);
    if (r->nout <= 0 || !r->d_hmax || bytes > copy_max) continue;
    add_pieces(pout, (const char*)r->ser.omax, r->d_hmax, bytes);
    add_pieces(pout, (const char*)r->ser.omin, r->d_hmin, bytes);
  }
  // descriptors, grouped by dtype
  std::vector<Group> groups;
  for (Req* r : reqs) {
    if (r->carry_only) continue;
    auto g = std::find_if(groups.begin(), groups.end(), [&](const Group& x) { return x.dt == r->dt; });
    if (g == groups.end()) {
      groups.push_back(Group{r->dt, {}});
      g = groups.end() - 1;
    }
    g->reqs.push_back(r);
  }
  // per dtype: descriptors, then one tile-prefix array per path (tile kernel
  // of lag 1..4, chunk kernel; the path from the batched plan's size
  // classes), built here on the host; after them the copy pieces.  One
  // upload of the whole image, then the gather kernel, one launch per path
  // present, and (below) the scatter kernel.
  constexpr int NP = mm::kBatchNP;
  struct GroupLaunch {
    int dt;
    int64_t S, run;
    size_t pos;
    int64_t acc[NP];
  };
  std::vector<GroupLaunch> gl;
  size_t total = 0;
  for (auto& g : groups) {
    gl.push_back(GroupLaunch{g.dt, (int64_t)g.reqs.size(), 0, total, {0, 0, 0, 0, 0}});
    total += g.reqs.size() * mm::series_bytes() + NP * (g.reqs.size() + 1) * sizeof(int64_t);
  }
  const size_t copy_at = (total + 15) & ~size_t(15);
  total = copy_at + (pin.size() + pout.size()) * sizeof(mm::CopyPiece);
  if (e == hipSuccess && total > L.desc_cap) {
    // the copy pieces need room: grow the lane's buffer (batches before
    // this one may still read the old one)
    e = hipStreamSynchronize(L.st);
    if (e == hipSuccess) {
      hipFree(L.desc);
      L.desc = nullptr;
      L.desc_cap = 0;
      e = hipMalloc((void**)&L.desc, 2 * total);
      if (e == hipSuccess) L.desc_cap = 2 * total;
    }
  }
  b->host.resize(total);
  for (size_t gi = 0; gi < groups.size(); ++gi) {
    GroupLaunch& G = gl[gi];
    const int64_t S = G.S;
    const mm::BatchPlan plan = mm::batch_plan_for(G.dt);
    G.run = (int64_t)plan.run_subtiles * mm::kTileOut;
    char* hd = b->host.data() + G.pos;
    int64_t* pre = (int64_t*)(hd + S * mm::series_bytes());
    for (int64_t k = 0; k < S; ++k) {
      Req* r = groups[gi].reqs[k];
      std::memcpy(hd + k * mm::series_bytes(), &r->ser, mm::series_bytes());
      for (int q = 0; q < NP; ++q) pre[q * (S + 1) + k] = G.acc[q];
      const int path = mm::batch_path(plan, r->ser.n, r->ser.w);
      if (path >= 0) G.acc[path] += mm::batch_tiles(path, r->ser.n, r->ser.w, G.run);
    }
    for (int q = 0; q < NP; ++q) pre[q * (S + 1) + S] = G.acc[q];
  }
  if (!pin.empty()) std::memcpy(b->host.data() + copy_at, pin.data(), pin.size() * sizeof(mm::CopyPiece));
  if (!pout.empty())
    std::memcpy(b->host.data() + copy_at + pin.size() * sizeof(mm::CopyPiece), pout.data(),
                pout.size() * sizeof(mm::CopyPiece));
  if (e == hipSuccess && total > 0) e = hipMemcpyAsync(L.desc, b->host.data(), total, hipMemcpyHostToDevice, L.st);
  if (e == hipSuccess)
    e = mm::launch_copy_pieces((const mm::CopyPiece*)(L.desc + copy_at), (int64_t)pin.size(), L.st);
  static const int kinds[NP] = {mm::kStratTile, mm::kStratTile2, mm::kStratTile3, mm::kStratTile4, mm::kStratChunk};
  for (const GroupLaunch& G : gl) {
    if (e != hipSuccess) break;
    char* dd = L.desc + G.pos;
    mm::JobArgs a;
    a.mode = 1;
    a.descs = dd;
    a.S = G.S;
    a.run = G.run;
    for (int q = 0; q < NP && e == hipSuccess; ++q) {
      if (G.acc[q] == 0) continue;
      a.pre = (const int64_t*)(dd + G.S * mm::series_bytes()) + q * (G.S + 1);
      if (kinds[q] == mm::kStratChunk) {
        if (mm::stream_lookback_state(L.st, std::min<int64_t>(G.acc[q], int64_t(1) << 20), &a.ring, &a.ring_lg,
                                      &a.ctl) != MAXMIN_OK) {
          e = hipErrorOutOfMemory;
          break;
        }
        chunked = true;
      }
      e = mm::launch_1d(G.dt, kinds[q], a, (int)std::min<int64_t>(G.acc[q], mm::grid_cap(G.dt, kinds[q])), L.st);
    }
  }
  // the chunk kernel flags a look-back wait that gave up in the lane's
  // control words: copy that word out with the batch, then clear it
  if (e == hipSuccess && seq == inject_err) {
    e = hipMemsetAsync(&L.ctl->err, 1, sizeof(uint32_t), L.st);
    chunked = true;
  }
  if (e == hipSuccess && chunked) {
    b->slot = L.next_slot++ % kErrSlots;
    L.h_err[b->slot] = 0;
    e = hipMemcpyAsync(&L.h_err[b->slot], &L.ctl->err, sizeof(uint32_t), hipMemcpyDeviceToHost, L.st);
    if (e == hipSuccess) e = hipMemsetAsync(&L.ctl->err, 0, sizeof(uint32_t), L.st);
  }
  // pushes that complete no window only roll their carry forward
  for (Req* r : reqs) {
    if (e != hipSuccess) break;
    if (r->carry_only && r->ser.carry) {
      mm::JobArgs a;
      a.a = r->ser.a;
      a.b = r->ser.b;
      a.na = r->ser.na;
      a.n = r->ser.n;
      a.w = r->ser.w;
      a.carry = r->ser.carry;
      e = mm::launch_carry_only(r->dt, a, L.st);
    }
  }
  // outputs: the scatter kernel's pieces, else copies
  if (e == hipSuccess)
    e = mm::launch_copy_pieces((const mm::CopyPiece*)(L.desc + copy_at) + pin.size(), (int64_t)pout.size(), L.st);
  for (Req* r : reqs) {
    if (e != hipSuccess) break;
    if (r->nout > 0 && (!r->d_hmax || r->nout * (int64_t)esize(r->dt) > copy_max)) {
      const size_t bytes = (size_t)r->nout * esize(r->dt);
      e = hipMemcpyAsync(r->h_max, r->ser.omax, bytes, hipMemcpyDeviceToHost, L.st);
      if (e == hipSuccess) e = hipMemcpyAsync(r->h_min, r->ser.omin, bytes, hipMemcpyDeviceToHost, L.st);
    }
  }
  if (e == hipSuccess) e = hipEventCreateWithFlags(&b->ev, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventRecord(b->ev, L.st);
  std::lock_guard<std::mutex> lk(mu);
  if (e != hipSuccess) {
    // nothing usable was produced: fail the batch's requests right away and
    // return each pushed stream to its state before the push (admission
    // advanced it; no later push of the stream has been admitted yet, since
    // admission and launch alternate on this thread), so the caller may
    // push the chunk again
    hipStreamSynchronize(L.st);
    for (Req* r : reqs) {
      if (r->kind == kPush) {
        auto it = streams.find(r->sid);
        if (it != streams.end()) {
          it->second.cur = 1 - it->second.cur;
          it->second.t -= r->n;
        }
      }
      arena.release(r->off, r->bytes);
      finish(r, MAXMIN_EDEVICE);
    }
    if (b->ev) hipEventDestroy(b->ev);
    delete b;
    cv_sched.notify_all();
    return;
  }
  ++n_batches;
  L.inflight.push_back(b);
  cv_poll.notify_all();
}

void maxmin_engine::scheduler_loop() {
  hipSetDevice(device);
  std::unique_lock<std::mutex> lk(mu);
  for (;;) {
    cv_sched.wait_for(lk, std::chrono::microseconds(500), [&] { return stop || !pending.empty(); });
    if (stop && pending.empty()) break;
    if (pending.empty()) continue;
    std::set<int64_t> used_sids;
    std::vector<std::vector<Req*>> per_lane(lanes.size());
    int64_t taken = 0;
    while (!pending.empty() && taken < max_batch * (int64_t)lanes.size()) {
      Req* r = pending.front();
      // a lane batch is full: stop here (its descriptors fill the lane buffer)
      bool full = false;
      for (auto& v : per_lane) full = full || (int64_t)v.size() >= max_batch;
      if (full) break;
      if (!admit(r, used_sids, per_lane)) break;
      pending.pop_front();
      ++taken;
    }
    peak_used = std::max(peak_used, arena.used);
    bool any = false;
    for (auto& v : per_lane) any = any || !v.empty();
    if (!any) {
      // head request waits for memory (or for its stream's previous push)
      cv_sched.wait_for(lk, std::chrono::microseconds(200));
      continue;
    }
    lk.unlock();
    for (size_t l = 0; l < per_lane.size(); ++l)
      if (!per_lane[l].empty()) launch((int)l, per_lane[l]);
    lk.lock();
  }
}

void maxmin_engine::poller_loop() {
  hipSetDevice(device);
  std::unique_lock<std::mutex> lk(mu);
  for (;;) {
    bool busy = false;
    for (auto& L : lanes) busy = busy || !L.inflight.empty();
    if (!busy) {
      if (stop && pending.empty()) break;
      cv_poll.wait_for(lk, std::chrono::milliseconds(2));
      continue;
    }
    bool progressed = false;
    for (auto& L : lanes) {
      while (!L.inflight.empty()) {
        Batch* b = L.inflight.front();
        if (hipEventQuery(b->ev) != hipSuccess) break;
        // a look-back wait that gave up leaves every output of the batch
        // suspect, and the carries its pushes wrote: fail them all and
        // mark those streams broken
        const bool bad = b->slot >= 0 && L.h_err[b->slot] != 0;
        for (Req* r : b->reqs) {
          arena.release(r->off, r->bytes);
          if (bad && r->kind == kPush) {
            auto it = streams.find(r->sid);
            if (it != streams.end()) it->second.broken = true;
          }
          if (!bad) elems_done += r->n;
          finish(r, bad ? MAXMIN_EDEVICE : MAXMIN_OK);
        }
        hipEventDestroy(b->ev);
        L.inflight.pop_front();
        delete b;
        progressed = true;
      }
    }
    if (progressed) cv_sched.notify_all();
    lk.unlock();
    std::this_thread::sleep_for(std::chrono::microseconds(20));
    lk.lock();
  }
}

extern "C" {

int maxmin_engine_create(int64_t hbm_budget_bytes, int n_lanes, int64_t max_batch, maxmin_engine_t** out) {
  if (!out) return mm::set_error(MAXMIN_EINVAL, "maxmin_engine_create: null out");
  *out = nullptr;
  if (hbm_budget_bytes < (1 << 20) || n_lanes < 1 || n_lanes > 16 || max_batch < 1)
    return mm::set_error(MAXMIN_EINVAL, "maxmin_engine_create: budget >= 1 MiB, 1..16 lanes, max_batch >= 1");
  std::unique_ptr<maxmin_engine> e(new maxmin_engine);
  hipGetDevice(&e->device);
  if (const char* c = getenv("MAXMIN_ENGINE_COPIES")) e->copy_kernels = strcmp(c, "memcpy") != 0;
  if (const char* c = getenv("MAXMIN_ENGINE_COPY_MAX")) {
    const long long v = atoll(c);
    if (v >= 0) e->copy_max = v;
  }
  if (const char* c = getenv("MAXMIN_ENGINE_MAX_PENDING")) {
    const long long v = atoll(c);
    if (v >= 1) e->max_pending = v;
  }
  if (const char* inj = getenv("MAXMIN_ENGINE_INJECT")) {
    long long k = 0;
    if (sscanf(inj, "launch:%lld", &k) == 1) e->inject_launch = k;
    if (sscanf(inj, "err:%lld", &k) == 1) e->inject_err = k;
  }
  if (hipMalloc((void**)&e->arena.base, (size_t)hbm_budget_bytes) != hipSuccess)
    return mm::set_error(MAXMIN_ENOMEM, "maxmin_engine_create: cannot allocate the HBM budget");
  e->arena.size = hbm_budget_bytes & ~int64_t(255);
  e->arena.free_[0] = e->arena.size;
  e->max_batch = max_batch;
  e->lanes.resize((size_t)n_lanes);
  for (auto& L : e->lanes) {
    if (hipStreamCreateWithFlags(&L.st, hipStreamNonBlocking) != hipSuccess) {
      for (auto& M : e->lanes)
        if (M.st) hipStreamDestroy(M.st);
      hipFree(e->arena.base);
      return mm::set_error(MAXMIN_EDEVICE, "maxmin_engine_create: hipStreamCreate failed");
    }
  }
  for (auto& L : e->lanes) {
    L.desc_cap = (size_t)max_batch * mm::series_bytes() + mm::kBatchNP * ((size_t)max_batch + 8) * sizeof(int64_t);
    uint64_t* ring;
    uint32_t lg;
    if (hipMalloc((void**)&L.desc, L.desc_cap) != hipSuccess ||
        hipHostMalloc((void**)&L.h_err, kErrSlots * sizeof(uint32_t), hipHostMallocDefault) != hipSuccess ||
        mm::stream_lookback_state(L.st, int64_t(1) << 20, &ring, &lg, &L.ctl) != MAXMIN_OK) {
      for (auto& M : e->lanes) {
        if (M.desc) hipFree(M.desc);
        if (M.h_err) hipHostFree(M.h_err);
        hipStreamDestroy(M.st);
      }
      hipFree(e->arena.base);
      return mm::set_error(MAXMIN_ENOMEM, "maxmin_engine_create: cannot allocate lane buffers");
    }
  }
  maxmin_engine* eng = e.release();
  eng->sched = std::thread([eng] { eng->scheduler_loop(); });
  eng->poller = std::thread([eng] { eng->poller_loop(); });
  *out = eng;
  return mm::set_error(MAXMIN_OK, "");
}

int maxmin_engine_open_stream(maxmin_engine_t* eng, int dtype, int64_t w, int64_t* stream_id) {
  if (!eng || !stream_id) return mm::set_error(MAXMIN_EINVAL, "maxmin_engine_open_stream: null argument");
  const size_t s = esize(dtype);
  if (!s || w < 1) return mm::set_error(MAXMIN_EINVAL, "maxmin_engine_open_stream: bad dtype or window");
  std::lock_guard<std::mutex> lk(eng->mu);
  EStream es;
  es.dt = dtype;
  es.w = w;
  const int64_t cb = 2 * Arena::up(std::max<int64_t>(1, w - 1) * (int64_t)s);
  es.off = eng->arena.alloc(cb);
  if (es.off < 0) return mm::set_error(MAXMIN_ENOMEM, "maxmin_engine_open_stream: budget exhausted");
  eng->reserved += cb;
  const int64_t sid = eng->next_sid++;
  es.lane = (int)(sid % (int64_t)eng->lanes.size());
  eng->streams[sid] = es;
  *stream_id = sid;
  return mm::set_error(MAXMIN_OK, "");
}

int maxmin_engine_close_stream(maxmin_engine_t* eng, int64_t stream_id) {
  if (!eng) return mm::set_error(MAXMIN_EINVAL, "maxmin_engine_close_stream: null engine");
  std::unique_lock<std::mutex> lk(eng->mu);
  auto it = eng->streams.find(stream_id);
  if (it == eng->streams.end()) return mm::set_error(MAXMIN_EINVAL, "maxmin_engine_close_stream: unknown stream");
  eng->cv_done.wait(lk, [&] { return it->second.queued == 0; });
  const int64_t cb = 2 * Arena::up(std::max<int64_t>(1, it->second.w - 1) * (int64_t)esize(it->second.dt));
  eng->arena.release(it->second.off, cb);
  eng->reserved -= cb;
  eng->streams.erase(it);
  return mm::set_error(MAXMIN_OK, "");
}

static int submit(maxmin_engine_t* eng, Req* r, int64_t* req_id) {
  if (eng->copy_kernels && r->n > 0) {
    // the batch's copy kernels reach pinned, mapped host buffers directly
    const void* di = mapped(r->h_in);
    void* dx = (void*)mapped(r->h_max);
    void* dn = (void*)mapped(r->h_min);
    if (di && dx && dn) {
      r->d_hin = (const char*)di;
      r->d_hmax = (char*)dx;
      r->d_hmin = (char*)dn;
    }
  }
  std::lock_guard<std::mutex> lk(eng->mu);
  if (eng->stop) {
    delete r;
    return mm::set_error(MAXMIN_EBUSY, "maxmin_engine: shutting down");
  }
  if ((int64_t)eng->pending.size() >= eng->max_pending) {
    ++eng->n_busy;
    delete r;
    return mm::set_error(MAXMIN_EBUSY, "maxmin_engine: admission queue full (back-pressure)");
  }
  if (r->kind == kPush) {
    auto it = eng->streams.find(r->sid);
    if (it == eng->streams.end()) {
      delete r;
      return mm::set_error(MAXMIN_EINVAL, "maxmin_engine_submit_push: unknown stream");
    }
    r->dt = it->second.dt;
    r->w = it->second.w;
    ++it->second.queued;
  }
  r->id = eng->next_id++;
  r->t_arrive = Clock::now();
  eng->pending.push_back(r);
  ++eng->n_submitted;
  ++eng->in_system;
  if (req_id) *req_id = r->id;
  eng->cv_sched.notify_one();
  return mm::set_error(MAXMIN_OK, "");
}

int maxmin_engine_submit_filter(maxmin_engine_t* eng, int dtype, const void* h_in, int64_t n, int64_t w, void* h_max,
                                void* h_min, int64_t* req_id) {
  if (!eng) return mm::set_error(MAXMIN_EINVAL, "maxmin_engine_submit_filter: null engine");
  if (!esize(dtype) || w < 1 || n < 0) return mm::set_error(MAXMIN_EINVAL, "maxmin_engine_submit_filter: bad dtype, n or w");
  if (n >= w && (!h_in || !h_max || !h_min)) return mm::set_error(MAXMIN_EINVAL, "maxmin_engine_submit_filter: null buffer");
  Req* r = new Req;
  r->kind = kFilter;
  r->dt = dtype;
  r->n = n;
  r->w = w;
  r->h_in = h_in;
  r->h_max = h_max;
  r->h_min = h_min;
  return submit(eng, r, req_id);
}

int maxmin_engine_submit_push(maxmin_engine_t* eng, int64_t stream_id, const void* h_chunk, int64_t m, void* h_max,
                              void* h_min, int64_t* req_id) {
  if (!eng || m < 0 || (m > 0 && (!h_chunk || !h_max || !h_min)))
    return mm::set_error(MAXMIN_EINVAL, "maxmin_engine_submit_push: bad argument");
  Req* r = new Req;
  r->kind = kPush;
  r->sid = stream_id;
  r->n = m;
  r->h_in = h_chunk;
  r->h_max = h_max;
  r->h_min = h_min;
  return submit(eng, r, req_id);
}

int maxmin_engine_poll(maxmin_engine_t* eng, int64_t* ids, int64_t* n_out, double* latency_s, int* status, int64_t cap,
                       int64_t* got) {
  if (!eng || !got || cap < 0) return mm::set_error(MAXMIN_EINVAL, "maxmin_engine_poll: bad argument");
  std::lock_guard<std::mutex> lk(eng->mu);
  int64_t k = 0;
  while (k < cap && !eng->done.empty()) {
    Req* r = eng->done.front();
    eng->done.pop_front();
    if (ids) ids[k] = r->id;
    if (n_out) n_out[k] = r->nout;
    if (latency_s) latency_s[k] = std::chrono::duration<double>(r->t_done - r->t_arrive).count();
    if (status) status[k] = r->status;
    --eng->in_system;
    delete r;
    ++k;
  }
  *got = k;
  return mm::set_error(MAXMIN_OK, "");
}

int maxmin_engine_drain(maxmin_engine_t* eng) {
  if (!eng) return mm::set_error(MAXMIN_EINVAL, "maxmin_engine_drain: null engine");
  std::unique_lock<std::mutex> lk(eng->mu);
  eng->cv_done.wait(lk, [&] { return eng->n_done == eng->n_submitted; });
  return mm::set_error(MAXMIN_OK, "");
}

int maxmin_engine_stats(maxmin_engine_t* eng, int64_t* out8) {
  if (!eng || !out8) return mm::set_error(MAXMIN_EINVAL, "maxmin_engine_stats: null argument");
  int64_t* out = out8;  // MAXMIN_ENGINE_STATS_LEN entries
  std::lock_guard<std::mutex> lk(eng->mu);
  out8[0] = eng->n_submitted;
  out8[1] = eng->n_done;
  out8[2] = eng->n_batches;
  out8[3] = eng->n_rejected;
  out8[4] = eng->elems_done;
  out8[5] = eng->arena.used;
  out8[6] = eng->peak_used;
  out8[7] = (int64_t)eng->pending.size();
  out[8] = eng->n_busy;
  return mm::set_error(MAXMIN_OK, "");
}

int maxmin_engine_destroy(maxmin_engine_t* eng) {
  if (!eng) return mm::set_error(MAXMIN_OK, "");
  {
    std::unique_lock<std::mutex> lk(eng->mu);
    eng->cv_done.wait(lk, [&] { return eng->n_done == eng->n_submitted; });
    eng->stop = true;
  }
  eng->cv_sched.notify_all();
  eng->cv_poll.notify_all();
  eng->sched.join();
  eng->poller.join();
  for (Req* r : eng->done) delete r;
  for (auto& L : eng->lanes) {
    hipStreamDestroy(L.st);
    hipFree(L.desc);
    hipHostFree(L.h_err);
  }
  hipFree(eng->arena.base);
  delete eng;
  return mm::set_error(MAXMIN_OK, "");
}

// Open-loop replay: submit request i at start + at_s[i] seconds (from one
// host thread), then return; completion is collected with poll/drain.
// kind[i] 0 = filter (dtype[i], n[i], w[i]), 1 = push on stream sid[i]
// (chunk of n[i] samples).
int maxmin_engine_replay(maxmin_engine_t* eng, int64_t count, const double* at_s, const int* kind, const int* dtype,
                         const int64_t* n, const int64_t* w, const int64_t* sid, const void* const* h_in,
                         void* const* h_max, void* const* h_min, int64_t* req_ids, double* lag_s) {
  if (!eng || count < 0 || (count > 0 && (!at_s || !kind || !n || !h_in || !h_max || !h_min)))
    return mm::set_error(MAXMIN_EINVAL, "maxmin_engine_replay: bad argument");
  const Clock::time_point t0 = Clock::now();
  for (int64_t i = 0; i < count; ++i) {
    const Clock::time_point due = t0 + std::chrono::duration_cast<Clock::duration>(std::chrono::duration<double>(at_s[i]));
    Clock::time_point now = Clock::now();
    if (now < due) {
      if (due - now > std::chrono::microseconds(200)) std::this_thread::sleep_until(due - std::chrono::microseconds(100));
      while ((now = Clock::now()) < due) {
      }
    }
    if (lag_s) lag_s[i] = std::chrono::duration<double>(now - due).count();
    int64_t id = 0;
    int rc = kind[i] == kFilter ? maxmin_engine_submit_filter(eng, dtype[i], h_in[i], n[i], w[i], h_max[i], h_min[i], &id)
                                : maxmin_engine_submit_push(eng, sid[i], h_in[i], n[i], h_max[i], h_min[i], &id);
    if (rc == MAXMIN_EBUSY && !eng->stop) id = -1;  // refused by back-pressure: keep replaying
    else if (rc != MAXMIN_OK) return rc;
    if (req_ids) req_ids[i] = id;
  }
  return mm::set_error(MAXMIN_OK, "");
}

}  // extern "C"
