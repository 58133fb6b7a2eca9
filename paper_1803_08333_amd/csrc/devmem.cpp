// Device memory cache of the library.
//
// Every device buffer the library owns (blocks, projector matrices, work
// vectors, scratch) is a DevBuf.  A released buffer goes onto a per-device
// free list instead of back to the driver; the next request of about the
// same size on that device takes it.  Building operators again and again on
// meshes of one size (a sweep over wavenumbers, or a new mesh of the same
// size each time) then maps no new memory after the first time.  A failed
// hipMalloc releases the whole cache and tries once more.
//
// Release waits for the device to be idle first (as hipFree would), so a
// block on the free list is never still read or written by queued work.
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>
#include <utility>

#include "internal.h"

namespace rfcmp {
namespace {

struct Cache {
  std::mutex mu;
  // (device, bytes) -> free blocks of that rounded size
  std::multimap<std::pair<int, size_t>, void*> blocks;
  size_t cached = 0;
};

Cache& cache() {
  static Cache* c = new Cache;  // never destroyed: the HIP runtime may be gone at exit
  return *c;
}

size_t rounded(size_t n) {
  const size_t g = n >= (size_t(1) << 20) ? (size_t(2) << 20) : 256;
  return (n + g - 1) / g * g;
}

}  // namespace

void* dev_alloc(size_t n, size_t* got, int* device) {
  const size_t r = rounded(n);
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return nullptr;
  Cache& c = cache();
  {
    std::lock_guard<std::mutex> g(c.mu);
    // smallest cached block of at least r bytes and at most r + r/8
    auto it = c.blocks.lower_bound({dev, r});
    if (it != c.blocks.end() && it->first.first == dev && it->first.second <= r + r / 8) {
      void* p = it->second;
      *got = it->first.second;
      c.cached -= it->first.second;
      c.blocks.erase(it);
      *device = dev;
      return p;
    }
  }
  void* p = nullptr;
  if (hipMalloc(&p, r) != hipSuccess) {
    (void)hipGetLastError();
    dev_cache_release();
    p = nullptr;
    if (hipMalloc(&p, r) != hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
  }
  *got = r;
  *device = dev;
  return p;
}

void dev_free(void* p, size_t bytes, int device) {
  if (!p) return;
  int cur = 0;
  (void)hipGetDevice(&cur);
  if (cur != device) (void)hipSetDevice(device);
  (void)hipDeviceSynchronize();
  if (cur != device) (void)hipSetDevice(cur);
  Cache& c = cache();
  std::lock_guard<std::mutex> g(c.mu);
  c.blocks.insert({{device, bytes}, p});
  c.cached += bytes;
}

size_t dev_cache_release() {
  Cache& c = cache();
  std::lock_guard<std::mutex> g(c.mu);
  size_t freed = 0;
  int cur = 0;
  (void)hipGetDevice(&cur);
  for (auto& kv : c.blocks) {
    (void)hipSetDevice(kv.first.first);
    (void)hipFree(kv.second);
    freed += kv.first.second;
  }
  (void)hipSetDevice(cur);
  c.blocks.clear();
  c.cached = 0;
  return freed;
}

size_t dev_cache_bytes() {
  Cache& c = cache();
  std::lock_guard<std::mutex> g(c.mu);
  return c.cached;
}

}  // namespace rfcmp

extern "C" rfcmp_status rfcmp_release_cached_memory(int64_t* freed_bytes) {
  const size_t f = rfcmp::dev_cache_release();
  if (freed_bytes) *freed_bytes = (int64_t)f;
  return RFCMP_OK;
}
