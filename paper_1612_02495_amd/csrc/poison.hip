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

}  // namespace

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
