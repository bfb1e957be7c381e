// Quiet-NaN fill of device workspaces (see poison.h).
#include "poison.h"

#include <cstdint>
#include <cstdlib>
#include <cstring>

namespace swept {
namespace {

template <typename W>
__global__ void __launch_bounds__(256) poison_kernel(W* __restrict__ p, int64_t count, W value) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < count; i += (int64_t)gridDim.x * 256) p[i] = value;
}

__global__ void nonfinite_reset_kernel(int* flag) { *flag = 0; }

template <typename T>
__global__ void __launch_bounds__(256) nonfinite_scan_kernel(const T* __restrict__ u, int64_t n, int* flag) {
  bool bad = false;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    bad = bad || !isfinite(u[i]);
  if (bad) atomicOr(flag, 1);
}

}  // namespace

hipError_t enqueue_nonfinite_check(const void* u, int64_t n, int elem_size, int* flag, hipStream_t st) {
  hipLaunchKernelGGL(nonfinite_reset_kernel, dim3(1), dim3(1), 0, st, flag);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || n <= 0) return e;
  const unsigned blocks = (unsigned)(n / 256 + 1 < 8192 ? n / 256 + 1 : 8192);
  if (elem_size == 8)
    hipLaunchKernelGGL(nonfinite_scan_kernel<double>, dim3(blocks), dim3(256), 0, st, static_cast<const double*>(u),
                       n, flag);
  else
    hipLaunchKernelGGL(nonfinite_scan_kernel<float>, dim3(blocks), dim3(256), 0, st, static_cast<const float*>(u), n,
                       flag);
  return hipGetLastError();
}

bool debug_poison_requested() {
  const char* v = std::getenv("SWEPT_DEBUG_POISON");
  return v && *v && std::strcmp(v, "0") != 0;
}

hipError_t poison_fill(void* p, size_t bytes, int elem_size, hipStream_t st) {
  if (!p || bytes == 0) return hipSuccess;
  if (elem_size == 8) {
    const int64_t count = (int64_t)(bytes / 8);
    const unsigned blocks = (unsigned)(count / 256 + 1 < 65536 ? count / 256 + 1 : 65536);
    hipLaunchKernelGGL(poison_kernel<uint64_t>, dim3(blocks), dim3(256), 0, st, static_cast<uint64_t*>(p), count,
                       (uint64_t)0x7FF8000000000000ull);
  } else {
    const int64_t count = (int64_t)(bytes / 4);
    const unsigned blocks = (unsigned)(count / 256 + 1 < 65536 ? count / 256 + 1 : 65536);
    hipLaunchKernelGGL(poison_kernel<uint32_t>, dim3(blocks), dim3(256), 0, st, static_cast<uint32_t*>(p), count,
                       (uint32_t)0x7FC00000u);
  }
  return hipGetLastError();
}

}  // namespace swept
