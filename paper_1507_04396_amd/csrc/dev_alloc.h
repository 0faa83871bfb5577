// Device memory of the library: hipMalloc/hipFree by default, or the caller's allocator once
// mmf_set_allocator installs one.  Each buffer remembers which allocator produced it, so changing
// the allocator later never frees a buffer through the wrong one.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>

namespace pmmf_alloc {

struct How {
  void (*release)(void*, void*, void*) = nullptr;  // null: the buffer came from hipMalloc
  void* ctx = nullptr;
  void* stream = nullptr;  // stream handed to the caller's allocator for this buffer
};

// nullptr on failure
void* alloc(size_t bytes, How* how);
// waits for the device first when the buffer came from the caller's allocator (as hipFree does),
// so memory that work on another stream still reads is never handed back early
void release(void* p, const How& how);

// the stream passed to the caller's allocator for allocations made by this thread in this scope
struct StreamScope {
  void* prev;
  explicit StreamScope(void* stream);
  ~StreamScope();
};

}  // namespace pmmf_alloc
