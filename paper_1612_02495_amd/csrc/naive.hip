// Classic decomposition (Sec. 4.4): one thread per grid point, one launch per
// sub-timestep, every value read from and written to global memory.  This is
// the baseline the swept rule is measured against; it shares the stencil
// arithmetic of stencil.h with the swept kernels, so both round identically.
#include "internal.h"

namespace swept {
namespace {

constexpr int kNaiveThreads = 256;

__device__ __forceinline__ int64_t wrap_once(int64_t i, int64_t n) {
  // n >= 4 and |offset| <= 2, so one correction suffices.
  return i < 0 ? i + n : (i >= n ? i - n : i);
}

__device__ __forceinline__ int64_t first_index() { return (int64_t)blockIdx.x * kNaiveThreads + threadIdx.x; }
__device__ __forceinline__ int64_t stride() { return (int64_t)gridDim.x * kNaiveThreads; }

template <typename T>
__global__ void __launch_bounds__(kNaiveThreads)
naive_heat_kernel(const T* __restrict__ in, T* __restrict__ out, int64_t n, Consts<T> k) {
  for (int64_t i = first_index(); i < n; i += stride())
    out[i] = heat_update(in[wrap_once(i - 1, n)], in[i], in[wrap_once(i + 1, n)], k);
}

// Insulated rod (Sec. 4.1): nodes 0 and n-1 take the mirror ghost about
// themselves, u_{-1} = u_1 and u_n = u_{n-2}.
template <typename T>
__global__ void __launch_bounds__(kNaiveThreads)
naive_heat_insulated_kernel(const T* __restrict__ in, T* __restrict__ out, int64_t n, Consts<T> k) {
  for (int64_t i = first_index(); i < n; i += stride()) {
    const T left = in[i == 0 ? 1 : i - 1];
    const T right = in[i == n - 1 ? n - 2 : i + 1];
    out[i] = heat_update(left, in[i], right, k);
  }
}

template <typename T>
__global__ void __launch_bounds__(kNaiveThreads)
naive_ks_predictor_kernel(const T* __restrict__ u, T* __restrict__ q, int64_t n, Consts<T> k) {
  for (int64_t i = first_index(); i < n; i += stride())
    q[i] = ks_predictor(u[wrap_once(i - 2, n)], u[wrap_once(i - 1, n)], u[i], u[wrap_once(i + 1, n)],
                        u[wrap_once(i + 2, n)], k);
}

template <typename T>
__global__ void __launch_bounds__(kNaiveThreads)
naive_ks_final_kernel(T* __restrict__ u, const T* __restrict__ q, int64_t n, Consts<T> k) {
  for (int64_t i = first_index(); i < n; i += stride())
    u[i] = ks_final(u[i], q[wrap_once(i - 2, n)], q[wrap_once(i - 1, n)], q[i], q[wrap_once(i + 1, n)],
                    q[wrap_once(i + 2, n)], k);
}

// One thread per point up to kNaiveMaxBlocks blocks (2^30 points); larger
// rings loop, so every grid size fits one launch.
constexpr int64_t kNaiveMaxBlocks = int64_t(1) << 22;

inline dim3 grid_for(int64_t n) {
  const int64_t blocks = (n + kNaiveThreads - 1) / kNaiveThreads;
  return dim3((unsigned)(blocks < kNaiveMaxBlocks ? blocks : kNaiveMaxBlocks));
}

}  // namespace

template <typename T>
hipError_t launch_naive_heat(const T* in, T* out, int64_t n, const Consts<T>& k, hipStream_t st) {
  hipLaunchKernelGGL(naive_heat_kernel<T>, grid_for(n), dim3(kNaiveThreads), 0, st, in, out, n, k);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_naive_heat_insulated(const T* in, T* out, int64_t n, const Consts<T>& k, hipStream_t st) {
  hipLaunchKernelGGL(naive_heat_insulated_kernel<T>, grid_for(n), dim3(kNaiveThreads), 0, st, in, out, n, k);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_naive_ks_predictor(const T* u, T* q, int64_t n, const Consts<T>& k, hipStream_t st) {
  hipLaunchKernelGGL(naive_ks_predictor_kernel<T>, grid_for(n), dim3(kNaiveThreads), 0, st, u, q, n, k);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_naive_ks_final(T* u, const T* q, int64_t n, const Consts<T>& k, hipStream_t st) {
  hipLaunchKernelGGL(naive_ks_final_kernel<T>, grid_for(n), dim3(kNaiveThreads), 0, st, u, q, n, k);
  return hipGetLastError();
}

template hipError_t launch_naive_heat<float>(const float*, float*, int64_t, const Consts<float>&, hipStream_t);
template hipError_t launch_naive_heat<double>(const double*, double*, int64_t, const Consts<double>&, hipStream_t);
template hipError_t launch_naive_heat_insulated<float>(const float*, float*, int64_t, const Consts<float>&,
                                                        hipStream_t);
template hipError_t launch_naive_heat_insulated<double>(const double*, double*, int64_t, const Consts<double>&,
                                                         hipStream_t);
template hipError_t launch_naive_ks_predictor<float>(const float*, float*, int64_t, const Consts<float>&, hipStream_t);
template hipError_t launch_naive_ks_predictor<double>(const double*, double*, int64_t, const Consts<double>&, hipStream_t);
template hipError_t launch_naive_ks_final<float>(float*, const float*, int64_t, const Consts<float>&, hipStream_t);
template hipError_t launch_naive_ks_final<double>(double*, const double*, int64_t, const Consts<double>&, hipStream_t);

}  // namespace swept
