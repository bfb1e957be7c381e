// Workspace poisoning for checking (SWEPT_DEBUG_POISON): every plan created
// while the variable is set to anything but "" or "0" fills its edge slots
// (and, for the adjoints, checkpoints and lambda slots) with quiet NaNs
// before each run, so an entry read before a phase wrote it turns the result
// into NaN instead of passing unnoticed.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>

namespace swept {

// Whether SWEPT_DEBUG_POISON asks for poisoned workspaces (read when a plan is created).
bool debug_poison_requested();

// Fill `bytes` of device memory at p with quiet NaNs of elem_size bytes (4 or
// 8; bytes a multiple of it) by a kernel on `st` -- no memset node, so the
// fill is safe inside a captured graph.
hipError_t poison_fill(void* p, size_t bytes, int elem_size, hipStream_t st);

}  // namespace swept
