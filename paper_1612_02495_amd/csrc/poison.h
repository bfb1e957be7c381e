// Workspace poisoning for checking (SWEPT_DEBUG_POISON): every plan created
// while the variable is set to anything but "" or "0" fills its edge slots
// (and, for the adjoints, checkpoints and lambda slots) with quiet NaNs
// before each run, so an entry read before a phase wrote it turns the result
// into NaN instead of passing unnoticed.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace swept {

// Whether SWEPT_DEBUG_POISON asks for poisoned workspaces (read when a plan is created).
bool debug_poison_requested();

// Fill `bytes` of device memory at p with quiet NaNs of elem_size bytes (4 or
// 8; bytes a multiple of it) by a kernel on `st` -- no memset node, so the
// fill is safe inside a captured graph.
hipError_t poison_fill(void* p, size_t bytes, int elem_size, hipStream_t st);

// Device side: fill `count` values of a workgroup's LDS buffer with quiet NaNs,
// thread `tid` of `nthr` taking every nthr-th value (the caller orders the
// fill before the buffer's first use).  Kernels call it at the start of each
// tile when the plan was created with SWEPT_DEBUG_POISON, so that a read of
// LDS that no store of the same tile preceded shows up as NaN as well.
template <typename T>
__device__ __forceinline__ T quiet_nan() {
  if constexpr (sizeof(T) == 8)
    return __longlong_as_double(0x7FF8000000000000ll);
  else
    return __int_as_float(0x7FC00000);
}
template <typename T>
__device__ __forceinline__ void poison_lds(T* p, int count, int tid, int nthr) {
  for (int i = tid; i < count; i += nthr) p[i] = quiet_nan<T>();
}

// Opt-in non-finite check (swept_plan_set_checks, swept_batch_set_checks):
// enqueue on `st` a reset of *flag followed by a scan of the n values at u
// (elem_size 4 or 8 bytes) that sets *flag when any of them is not finite.
// Kernels only (no memset), so the check may be part of a captured graph.
hipError_t enqueue_nonfinite_check(const void* u, int64_t n, int elem_size, int* flag, hipStream_t st);

}  // namespace swept
