// Process-wide cache of device memory blocks, per device.
//
// A factorization allocates and releases scratch level by level (hundreds of
// 256 MiB chunks for a 4M-unknown problem) and a solve allocates its Krylov
// basis every call.  Going to hipMalloc/hipFree for each costs host time,
// makes every release synchronise the device, and makes the driver clear
// fresh pages.  Released blocks are kept here instead and handed out again
// to a request of the same rounded size (best fit, at most twice the size
// asked for).  Sizes are rounded up to 2 MiB.  The cache holds at most
// SPAND_POOL_MB MiB per process (default: three quarters of the first
// device's memory); beyond that blocks go back to the driver, and so does the whole
// cache before a new block would leave less than 8 GiB free.
// spand_pool_trim() returns every cached block.
//
// A block may be released only once no queued work uses it: every caller
// synchronises the stream that used the block before releasing it.
#include <algorithm>
#include <chrono>
#include <cstdlib>
#include <map>
#include <mutex>
#include <vector>

#include "internal.h"

namespace spand {

namespace {
struct Pool {
  std::mutex mu;
  std::map<int, std::multimap<size_t, void *>> free;   // device -> size -> block
  size_t cached = 0;
};
Pool &pool() {
  static Pool *p = new Pool();    // never destroyed: usable from other static destructors
  return *p;
}
size_t pool_cap() {
  static const size_t cap = [] {
    const char *e = std::getenv("SPAND_POOL_MB");
    if (e) {
      const long long mb = std::atoll(e);
      return size_t(mb < 0 ? 0 : mb) << 20;
    }
    // three quarters of the device memory: a factorization's transient
    // scratch plus its stored factor stay cached across repeated
    // factorizations (FP64 at 4M unknowns peaks near 150 GB); the headroom
    // rule below hands the cache back when others need the memory
    size_t fr = 0, tot = 0;
    if (hipMemGetInfo(&fr, &tot) != hipSuccess || tot == 0) return size_t(65536) << 20;
    return tot / 4 * 3;
  }();
  return cap;
}
constexpr size_t kRound = size_t(2) << 20;
constexpr size_t kHeadroom = size_t(8) << 30;
thread_local double t_driver_ms = 0.0;     // this thread's time in hipMalloc/hipFree
struct DriverTimer {
  std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();
  ~DriverTimer() {
    t_driver_ms += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  }
};
}  // namespace

double pool_driver_ms() { return t_driver_ms; }

size_t pool_round(size_t bytes) { return (std::max<size_t>(bytes, 1) + kRound - 1) / kRound * kRound; }

int pool_alloc(void **p, size_t bytes, size_t *got) {
  const size_t sz = pool_round(bytes);
  int dev = 0;
  SP_HIP(hipGetDevice(&dev));
  {
    Pool &P = pool();
    std::lock_guard<std::mutex> lk(P.mu);
    auto &fl = P.free[dev];
    auto it = fl.lower_bound(sz);
    if (it != fl.end() && it->first <= 2 * sz) {
      *p = it->second;
      *got = it->first;
      P.cached -= it->first;
      fl.erase(it);
      return SPAND_OK;
    }
  }
  DriverTimer tm;
  // keep headroom on the device for allocations the library does not see
  // (the runtime's own buffers, the caller's tensors): when a new block would
  // leave less than kHeadroom free, the cached blocks go back to the driver
  // first, all at once (the first release waits for the device; the others
  // then cost nothing more)
  {
    size_t fr = 0, tot = 0;
    if (hipMemGetInfo(&fr, &tot) == hipSuccess && fr < sz + kHeadroom && pool_cached_bytes() > 0)
      pool_trim();
  }
  hipError_t e = hipMalloc(p, sz);
  if (e != hipSuccess) {
    // give the cache back to the driver and try once more
    pool_trim();
    e = hipMalloc(p, sz);
  }
  if (e != hipSuccess) {
    *p = nullptr;
    set_error("hipMalloc(%zu bytes) failed: %s", sz, hipGetErrorString(e));
    return SPAND_ENOMEM;
  }
  *got = sz;
  return SPAND_OK;
}

// `bytes` is the size pool_alloc reported in *got.
void pool_release(void *p, size_t bytes) {
  if (!p) return;
  const size_t sz = bytes;
  int dev = 0;
  hipPointerAttribute_t at;
  if (hipPointerGetAttributes(&at, p) == hipSuccess) dev = at.device;
  else (void)hipGetDevice(&dev);
  Pool &P = pool();
  {
    std::lock_guard<std::mutex> lk(P.mu);
    if (P.cached + sz <= pool_cap()) {
      P.free[dev].emplace(sz, p);
      P.cached += sz;
      return;
    }
  }
  DriverTimer tm;
  (void)hipFree(p);
}

void pool_trim() {
  Pool &P = pool();
  std::lock_guard<std::mutex> lk(P.mu);
  int cur = 0;
  (void)hipGetDevice(&cur);
  for (auto &d : P.free) {
    (void)hipSetDevice(d.first);
    for (auto &b : d.second) (void)hipFree(b.second);
    d.second.clear();
  }
  (void)hipSetDevice(cur);
  P.cached = 0;
}

size_t pool_cached_bytes() {
  Pool &P = pool();
  std::lock_guard<std::mutex> lk(P.mu);
  return P.cached;
}

// ----------------------------------------------------------------- timing events
// A factorization times its phases and kernel batches with a few hundred
// events; creating each costs host time on the path that plans the upper
// levels, so finished events are kept per device and handed out again.
namespace {
struct EventCache {
  std::mutex mu;
  std::map<int, std::vector<hipEvent_t>> free;
};
EventCache &event_cache() {
  static EventCache *c = new EventCache();
  return *c;
}
constexpr size_t kEventCap = 8192;
}  // namespace

int event_get(hipEvent_t *e) {
  int dev = 0;
  SP_HIP(hipGetDevice(&dev));
  {
    EventCache &C = event_cache();
    std::lock_guard<std::mutex> lk(C.mu);
    auto &v = C.free[dev];
    if (!v.empty()) {
      *e = v.back();
      v.pop_back();
      return SPAND_OK;
    }
  }
  SP_HIP(hipEventCreate(e));
  return SPAND_OK;
}

void event_put(hipEvent_t e) {
  if (!e) return;
  int dev = 0;
  (void)hipGetDevice(&dev);
  EventCache &C = event_cache();
  {
    std::lock_guard<std::mutex> lk(C.mu);
    auto &v = C.free[dev];
    if (v.size() < kEventCap) {
      v.push_back(e);
      return;
    }
  }
  (void)hipEventDestroy(e);
}

}  // namespace spand
