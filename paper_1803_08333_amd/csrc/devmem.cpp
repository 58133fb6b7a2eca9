// Device memory of the library.
//
// Every device buffer the library owns (blocks, projector matrices, work
// vectors, scratch) is a DevBuf.  With an allocator registered by
// rfcmp_set_allocator (for instance a framework's caching allocator) every
// block comes from it and goes back to it.  Otherwise the library keeps its
// own cache over hipMalloc: a released buffer goes onto a per-device free
// list instead of back to the driver, and the next request of about the same
// size on that device takes it.  Building operators again and again on meshes
// of one size (a sweep over wavenumbers, or a new mesh of the same size each
// time) then maps no new memory after the first time.  A failed hipMalloc
// releases the whole cache and tries once more.
//
// Release waits for the device to be idle first (as hipFree would), so a
// block handed back is never still read or written by queued work.
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

struct Hook {
  std::mutex mu;
  rfcmp_alloc_fn alloc_fn = nullptr;
  rfcmp_free_fn free_fn = nullptr;
  void* ctx = nullptr;
};

Hook& hook() {
  static Hook* h = new Hook;
  return *h;
}

size_t rounded(size_t n) {
  const size_t g = n >= (size_t(1) << 20) ? (size_t(2) << 20) : 256;
  return (n + g - 1) / g * g;
}

}  // namespace

void* dev_alloc(size_t n, size_t* got, int* device, AllocOrigin* origin) {
  const size_t r = rounded(n);
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return nullptr;
  rfcmp_alloc_fn afn = nullptr;
  AllocOrigin from;
  {
    Hook& h = hook();
    std::lock_guard<std::mutex> g(h.mu);
    afn = h.alloc_fn;
    from.free_fn = h.free_fn;
    from.ctx = h.ctx;
  }
  if (afn) {
    void* p = afn(r, nullptr, from.ctx);
    if (!p) return nullptr;
    *got = r;
    *device = dev;
    *origin = from;
    return p;
  }
  *origin = AllocOrigin{};
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

void dev_free(void* p, size_t bytes, int device, const AllocOrigin& origin) {
  if (!p) return;
  int cur = 0;
  (void)hipGetDevice(&cur);
  if (cur != device) (void)hipSetDevice(device);
  (void)hipDeviceSynchronize();
  if (origin.free_fn) origin.free_fn(p, bytes, nullptr, origin.ctx);
  if (cur != device) (void)hipSetDevice(cur);
  if (origin.free_fn) return;
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

extern "C" rfcmp_status rfcmp_set_allocator(rfcmp_alloc_fn alloc_fn, rfcmp_free_fn free_fn, void* ctx) {
  rfcmp::clear_error();
  if ((alloc_fn == nullptr) != (free_fn == nullptr)) {
    rfcmp::set_error("rfcmp_set_allocator: give both functions or neither");
    return RFCMP_E_ARG;
  }
  rfcmp::Hook& h = rfcmp::hook();
  std::lock_guard<std::mutex> g(h.mu);
  h.alloc_fn = alloc_fn;
  h.free_fn = free_fn;
  h.ctx = alloc_fn ? ctx : nullptr;
  return RFCMP_OK;
}

extern "C" rfcmp_status rfcmp_release_cached_memory(int64_t* freed_bytes) {
  const size_t f = rfcmp::dev_cache_release();
  if (freed_bytes) *freed_bytes = (int64_t)f;
  return RFCMP_OK;
}
