// common.hpp -- shared definitions of the HIP implementation of knnjoin.h.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <stdexcept>
#include <string>

#include "../../include/knnjoin.h"

namespace knn {

// Error carrying a KNN_E* code; converted to a return code at the ABI edge.
struct Error : std::runtime_error {
  int code;
  Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

void set_last_error(const std::string& msg);

#define KNN_HIP(call)                                                          \
  do {                                                                         \
    hipError_t e_ = (call);                                                    \
    if (e_ != hipSuccess) {                                                    \
      int code_ = (e_ == hipErrorOutOfMemory) ? KNN_ENOMEM : KNN_EDEVICE;      \
      throw ::knn::Error(code_, std::string(#call) + ": " + hipGetErrorString(e_) + \
                                    " (" + __FILE__ + ":" + std::to_string(__LINE__) + ")"); \
    }                                                                          \
  } while (0)

#define KNN_CHECK(cond, code, msg)                                             \
  do {                                                                         \
    if (!(cond)) throw ::knn::Error((code), (msg));                            \
  } while (0)

// Launch-error check after a kernel launch.
#define KNN_LAUNCHED() KNN_HIP(hipGetLastError())

constexpr int kWave = 64;

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Device memory cache, per device.  Requests are rounded up to 256 bytes
// (below 1 MiB) or to whole MiB.  A released block goes back to the cache
// and is handed out again to a rounded request of at least 4/5 of its size,
// so a buffer of b requested bytes holds at most 1.25 (b + 1 MiB).  Every
// user releases memory only after the device work that used it has finished
// (the library's calls return after their work; an asynchronous graph replay
// is waited for before its scratch is released), so a reused block needs no
// stream ordering.  At most KNN_DEVICE_CACHE_BYTES (default 32 GiB) per device
// is kept; the cache is emptied and the allocation retried when hipMalloc
// runs out of memory.
constexpr double kPoolSlack = 1.25;                  // capacity / rounded request, at most
constexpr size_t kPoolRound = (size_t)1 << 20;       // rounding of large requests
void* device_acquire(size_t bytes, int* device, size_t* capacity);
void device_release(void* p, int device, size_t capacity);

// Bump allocation from a fixed device region instead of the cache: while an
// ArenaScope is alive on a thread, device_acquire on that thread hands out
// consecutive 256-byte aligned pieces of [base, base + size) (KNN_ENOMEM once
// they run out), marks them with device kArenaDevice, and device_release
// ignores them; pinned host buffers (HostBuf) come from a static per-thread
// block.  No HIP allocation is made in the scope.
constexpr int kArenaDevice = -2;
constexpr size_t kArenaHostBytes = 8192;
struct ArenaScope {
  char* base;
  size_t size;
  size_t used = 0;
  ArenaScope* prev;
  ArenaScope(void* base_, size_t size_);
  ~ArenaScope();
  ArenaScope(const ArenaScope&) = delete;
  ArenaScope& operator=(const ArenaScope&) = delete;
};
bool arena_active();
void* arena_host_block();  // kArenaHostBytes of host memory owned by the thread

// Device buffer owned by RAII (memory from the device cache).
template <class T>
struct DevBuf {
  T* p = nullptr;
  size_t n = 0;
  int dev = -1;
  DevBuf() = default;
  explicit DevBuf(size_t count) { alloc(count); }
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  DevBuf(DevBuf&& o) noexcept : p(o.p), n(o.n), dev(o.dev) {
    o.p = nullptr;
    o.n = 0;
  }
  DevBuf& operator=(DevBuf&& o) noexcept {
    if (this != &o) {
      release();
      p = o.p;
      n = o.n;
      dev = o.dev;
      o.p = nullptr;
      o.n = 0;
    }
    return *this;
  }
  ~DevBuf() { release(); }
  void alloc(size_t count) {
    release();
    if (count == 0) count = 1;
    size_t cap = 0;
    p = static_cast<T*>(device_acquire(count * sizeof(T), &dev, &cap));
    n = cap / sizeof(T);
  }
  // Grow to at least `count` elements (contents not preserved); true when
  // the buffer was (re)allocated.
  bool reserve(size_t count) {
    if (count > n || p == nullptr) {
      alloc(count);
      return true;
    }
    return false;
  }
  void release() {
    if (p) device_release(p, dev, n * sizeof(T));
    p = nullptr;
    n = 0;
  }
  size_t bytes() const { return n * sizeof(T); }
};

// Pinned host memory (for the small per-level read-backs: a copy into
// pinned memory avoids the staging of pageable destinations).
template <class T>
struct HostBuf {
  T* p = nullptr;
  size_t n = 0;
  HostBuf() = default;
  HostBuf(const HostBuf&) = delete;
  HostBuf& operator=(const HostBuf&) = delete;
  bool borrowed = false;  // the thread's arena host block, never freed here
  ~HostBuf() {
    if (p && !borrowed) (void)hipHostFree(p);
  }
  void reserve(size_t count) {
    if (p && count <= n) return;
    if (p && !borrowed) (void)hipHostFree(p);
    p = nullptr;
    n = 0;
    borrowed = false;
    if (arena_active()) {
      KNN_CHECK(count * sizeof(T) <= kArenaHostBytes, KNN_EINTERNAL,
                "host read-back buffer above the arena's host block");
      p = static_cast<T*>(arena_host_block());
      borrowed = true;
      n = count;
      return;
    }
    KNN_HIP(hipHostMalloc(reinterpret_cast<void**>(&p), count * sizeof(T), hipHostMallocDefault));
    n = count;
  }
};

}  // namespace knn
