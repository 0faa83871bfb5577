// Device memory of the library: hipMalloc by default, with released blocks kept for reuse, or the
// caller's allocator once mmf_set_allocator installs one.  Each buffer remembers which allocator produced it, so changing
// the allocator later never frees a buffer through the wrong one.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>

namespace pmmf_alloc {

struct How {
  void (*release)(void*, void*, void*) = nullptr;  // null: the buffer came from the default allocator
  void* ctx = nullptr;
  void* stream = nullptr;  // stream handed to the caller's allocator for this buffer
};

// nullptr on failure
void* alloc(size_t bytes, How* how);
// waits for the device first when the buffer came from the caller's allocator (as hipFree does),
// so memory that work on another stream still reads is never handed back early; a default block
// is kept, and reused by another stream only after the device has been synchronized
void release(void* p, const How& how);
// frees the kept blocks of the default allocator (waits for the device)
void trim();

// the stream passed to the caller's allocator for allocations made by this thread in this scope
struct StreamScope {
  void* prev;
  explicit StreamScope(void* stream);
  ~StreamScope();
};

}  // namespace pmmf_alloc
