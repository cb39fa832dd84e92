// Device memory of the problem contexts: hipMalloc, or one block per
// context while an arena is installed on the allocating thread.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>

namespace ibim {

// Device arenas.  hipFree waits for all work on the device, so a context
// whose arrays are freed one by one while other streams keep the device busy
// waits that long once per array.  While an arena is installed on a thread
// (ArenaScope), that thread's device_alloc calls (dalloc of the contexts) are
// carved out of one block (256-byte aligned; what does not fit goes to
// hipMalloc), device_free (dfree) leaves pointers inside a live block alone,
// and arena_release frees the block with one hipFree once nothing in it is
// used any more.
struct DeviceArena {
  char* base = nullptr;
  size_t size = 0, top = 0;
  size_t outside = 0;  // bytes that did not fit and came from hipMalloc
};
// Allocates and registers a block of `bytes` (a->base stays null on failure).
hipError_t arena_create(DeviceArena* a, size_t bytes);
// Unregisters the block, then frees it; a no-op without a block.
void arena_release(DeviceArena* a);
hipError_t device_alloc(void** p, size_t bytes);  // the thread's arena, else hipMalloc
void device_free(void* p);                        // hipFree unless inside a live arena

struct ArenaScope {
  DeviceArena* prev;
  explicit ArenaScope(DeviceArena* a);
  ~ArenaScope();
};

}  // namespace ibim
