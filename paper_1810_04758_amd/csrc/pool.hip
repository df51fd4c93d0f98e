// pool.hip -- the device memory cache behind DevBuf (see common.hpp).
#include <algorithm>
#include <cstdlib>
#include <string>
#include <map>
#include <mutex>

#include "common.hpp"

namespace knn {

namespace {

struct Pool {
  std::multimap<size_t, void*> free;  // capacity -> block
  size_t cached = 0;
};

std::mutex g_mu;
std::map<int, Pool> g_pools;

size_t cache_limit() {
  static const size_t lim = [] {
    const char* e = std::getenv("KNN_DEVICE_CACHE_BYTES");
    return e ? (size_t)std::strtoull(e, nullptr, 10) : (size_t)32 << 30;
  }();
  return lim;
}

// Requests are rounded so that sizes that differ a little share blocks.
size_t round_up(size_t b) {
  const size_t g = b < ((size_t)1 << 20) ? 256 : ((size_t)1 << 20);
  return (b + g - 1) / g * g;
}

void drain_locked(Pool& pl) {
  for (auto& kv : pl.free) (void)hipFree(kv.second);
  pl.free.clear();
  pl.cached = 0;
}

thread_local ArenaScope* t_arena = nullptr;
alignas(256) thread_local unsigned char t_arena_host[kArenaHostBytes];

}  // namespace

ArenaScope::ArenaScope(void* base_, size_t size_)
    : base(static_cast<char*>(base_)), size(size_), prev(t_arena) {
  t_arena = this;
}

ArenaScope::~ArenaScope() { t_arena = prev; }

bool arena_active() { return t_arena != nullptr; }

void* arena_host_block() { return t_arena_host; }

void* device_acquire(size_t bytes, int* device, size_t* capacity) {
  if (ArenaScope* a = t_arena) {
    const size_t b = (std::max<size_t>(bytes, 1) + 255) / 256 * 256;
    if (b > a->size - a->used)
      throw Error(KNN_ENOMEM, "no-allocation join: its buffers need more than the " +
                                  std::to_string(a->size) + "-byte scratch area");
    void* p = a->base + a->used;
    a->used += b;
    *device = kArenaDevice;
    *capacity = b;
    return p;
  }
  const size_t want = round_up(bytes == 0 ? 1 : bytes);
  int dev = 0;
  KNN_HIP(hipGetDevice(&dev));
  *device = dev;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    Pool& pl = g_pools[dev];
    auto it = pl.free.lower_bound(want);
    if (it != pl.free.end() && it->first <= want + want / 4) {
      void* p = it->second;
      *capacity = it->first;
      pl.cached -= it->first;
      pl.free.erase(it);
      return p;
    }
  }
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, want);
  if (e == hipErrorOutOfMemory) {
    (void)hipGetLastError();
    {
      std::lock_guard<std::mutex> lk(g_mu);
      drain_locked(g_pools[dev]);
    }
    e = hipMalloc(&p, want);
  }
  KNN_HIP(e);
  *capacity = want;
  return p;
}

void device_release(void* p, int device, size_t capacity) {
  if (!p || device == kArenaDevice) return;  // arena pieces are not the cache's
  std::lock_guard<std::mutex> lk(g_mu);
  Pool& pl = g_pools[device];
  if (pl.cached + capacity > cache_limit()) {
    (void)hipFree(p);
    return;
  }
  pl.free.emplace(capacity, p);
  pl.cached += capacity;
}

}  // namespace knn
