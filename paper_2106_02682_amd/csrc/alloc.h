// Device memory of the library's objects: hipMalloc / hipFree by default, or the caller's allocator
// (vemb_set_allocator, e.g. torch's caching allocator).  Every object keeps the allocator in effect at
// its creation and returns its memory through it.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <vector>

#include "common.h"

namespace vemb {

struct Allocator {
  vemb_alloc_fn alloc = nullptr;  // null: hipMalloc / hipFree
  vemb_free_fn free = nullptr;
  void* ctx = nullptr;
};

// The allocator in effect now (a copy), and the count of live objects that hold one.
Allocator current_allocator();
void object_created();
void object_destroyed();

inline void* device_alloc(const Allocator& a, size_t bytes) {
  if (bytes == 0) bytes = 16;
  if (a.alloc) return a.alloc(bytes, a.ctx);
  void* p = nullptr;
  return hipMalloc(&p, bytes) == hipSuccess ? p : nullptr;
}
inline void device_free(const Allocator& a, void* p) {
  if (!p) return;
  if (a.free)
    a.free(p, a.ctx);
  else
    hipFree(p);
}

// The device allocations of one object, released together.
struct DeviceMemory {
  Allocator a = current_allocator();
  std::vector<void*> ptrs;
  void* get(size_t bytes) {
    void* p = device_alloc(a, bytes);
    if (p) ptrs.push_back(p);
    return p;
  }
  void release() {
    for (void* p : ptrs) device_free(a, p);
    ptrs.clear();
  }
};

}  // namespace vemb
