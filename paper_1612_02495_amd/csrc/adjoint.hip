// Swept adjoint of the periodic heat FTCS scheme: gradients of
// J = 1/2 ||u_T - y||^2 with respect to u_0 and to the diffusivity alpha of
// every grid in a batch, by a reverse swept sweep that recomputes each swept
// cycle from its checkpointed edge states instead of storing every step.
//
// Scheme (Eq. HeatDisc, periodic): u_{m+1} = A u_m, A = Fo (S- + S+) + (1-2Fo) I,
// Fo = alpha dt/dx^2.  Reverse mode: lambda_T = dJ/du_T (given), lambda_m =
// A^T lambda_{m+1} = A lambda_{m+1} (A is symmetric: the same gather stencil
// and operation order as the forward), dJ/du_0 = lambda_0, and
// dJ/dalpha = (dt/dx^2) sum_m sum_i lambda_{m+1,i} (u_{m,i-1} + u_{m,i+1} - 2 u_{m,i}).
//
// Tiling.  Tiles of w = 64 points, one point per thread of a 64-thread block,
// full (pure) phases of h = 32 steps; the T mod 32 leading steps run with the
// classic scheme and keep their states.  Forward: phase p writes its edge
// slots out of place, into checkpoint p.  Reverse, for p = K .. 0, one fused
// launch per phase: every tile
//   1. recomputes its forward region (V then Lambda) from checkpoint p-1,
//      keeping every tier in LDS;
//   2. walks lambda down through the same region: its Lambda part first,
//      taking the lambda values of later regions just outside each tier from
//      lambda slots, then its V part, handing the two outermost values of each
//      gap tier on to the previous phase through the same slots;
//   3. adds lambda(x,t) (u(x-1,t-1) + u(x+1,t-1) - 2u(x,t-1)) over its points.
// The lambda slots mirror the forward edge slots: position-major [p][t & 1],
// (h+1) positions per side, updated in place by the tile that owns them.
// dJ/dalpha is summed per tile in phase order, then over tiles and remainder
// blocks in a fixed order: the result does not depend on scheduling.
#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "internal.h"
#include "swept.h"

namespace swept {
namespace adj {

constexpr int kW = 64;
constexpr int kH = 32;  // w / 2: tiers of a full triangle
constexpr int kA = 32;  // inner seam
constexpr int kSL = kW + 2;
constexpr int kRemThreads = 256;

__global__ void consts_kernel(const double* __restrict__ alpha, int batch, double dt, double dx,
                              Consts<double>* __restrict__ k) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= batch) return;
  // same formulas as swept_plan_create (Sec. 4.1, Sec. 5)
  const double fo = (alpha[b] * dt) / (dx * dx);
  Consts<double> c{};
  c.fo = fo;
  c.c = 1.0 - 2.0 * fo;
  k[b] = c;
}

// Row of tile points computed at diamond tier d (V part d <= h, Lambda d > h).
__device__ __forceinline__ bool in_row(int x, int d) {
  if (d < kH) return x >= kA - d && x < kA + d;
  if (d == kH) return x >= 0 && x < kW;
  return x >= d - kH && x < kW - d + kH;
}

// MODE 0: forward phase writing checkpoint slots (or u_T); MODE 1: fused adjoint.
template <int MODE>
__global__ void __launch_bounds__(kW)
region_kernel(const double* __restrict__ ustart, double* __restrict__ uT, const double* __restrict__ ck_in,
              double* __restrict__ ck_out, const double* __restrict__ gT, double* lam_slots, double* __restrict__ g_ur,
              double* __restrict__ partial, const Consts<double>* __restrict__ kb, int64_t n, int64_t nt, int p,
              int K) {
  constexpr int NROW = MODE ? 2 * kH + 1 : 2;
  __shared__ double hist[NROW][kW + 2];  // column x + 1, x in [-1, w]
  __shared__ double sin_l[kSL], sin_r[kSL];
  __shared__ double lam[2][kW + 2];
  __shared__ double lin_l[kSL], lin_r[kSL];
  __shared__ double red[kW];

  const int x = threadIdx.x;
  const int64_t b = blockIdx.x / nt;
  const int64_t j = blockIdx.x % nt;
  const Consts<double> k = kb[b];
  const int hv = p == 0 ? 0 : kH;
  const int hl = p == K ? 0 : kH;
  const int par = p & 1;
  const int64_t origin = j * kW + (par ? kA : 0);
  const int64_t base = b * 2 * nt * kSL;
  const int64_t sL = par ? (nt + j) * kSL : j * kSL;
  const int64_t sR = par ? ((j + 1) % nt) * kSL : (nt + j) * kSL;
  int64_t gx = origin + x;
  if (gx >= n) gx -= n;
  const int64_t gidx = b * n + gx;
#define ROW(d) (MODE ? (d) : ((d)&1))

  // ------------------------------------------------ forward recompute --
  if (hv == 0) {
    hist[ROW(kH)][x + 1] = ustart[gidx];
  } else {
    for (int i = x; i < kSL; i += kW) {
      sin_l[i] = ck_in[base + sL + i];
      sin_r[i] = ck_in[base + sR + i];
    }
    __syncthreads();
    for (int d = 0; d <= kH; ++d) {
      if (d > 0 && in_row(x, d))
        hist[ROW(d)][x + 1] = heat_update(hist[ROW(d - 1)][x], hist[ROW(d - 1)][x + 1], hist[ROW(d - 1)][x + 2], k);
      if (d < kH && x < 4) {
        // edge bands of tier d: [a-d-2, a-d) from the left slot, [a+d, a+d+2) from the right
        const int pos = x < 2 ? kA - d - 2 + x : kA + d + (x - 2);
        hist[ROW(d)][pos + 1] = x < 2 ? sin_l[2 * (pos + 1) + (d & 1)] : sin_r[2 * (pos - kA) + (d & 1)];
      }
      __syncthreads();
    }
  }
  if (hl > 0) {
    __syncthreads();
    for (int m = 0; m < kH; ++m) {
      const int d = kH + m;
      if (m > 0 && in_row(x, d))
        hist[ROW(d)][x + 1] = heat_update(hist[ROW(d - 1)][x], hist[ROW(d - 1)][x + 1], hist[ROW(d - 1)][x + 2], k);
      __syncthreads();
      if constexpr (MODE == 0) {
        if (x < 4) {
          const int pos = x < 2 ? m + x : kW - m - 2 + (x - 2);
          const double v = hist[ROW(d)][pos + 1];
          if (x < 2)
            ck_out[base + sL + 2 * pos + (m & 1)] = v;
          else
            ck_out[base + sR + 2 * (pos - kA + 1) + (m & 1)] = v;
        }
      }
    }
  } else if constexpr (MODE == 0) {
    uT[gidx] = hist[ROW(kH)][x + 1];
  }
  if constexpr (MODE == 0) return;

  // --------------------------------------------------- adjoint sweep --
  __syncthreads();
  for (int i = x; i < kSL; i += kW) {
    lin_l[i] = lam_slots[base + sL + i];
    lin_r[i] = lam_slots[base + sR + i];
  }
  __syncthreads();
  // lambda values of later regions just outside Lambda tier t = h + m
  auto incoming = [&](double* row, int t) {
    const int m = t - kH;
    if (x < 4) {
      const int pos = x < 2 ? m - 2 + x : kW - m + (x - 2);
      row[pos + 1] = x < 2 ? lin_l[2 * (pos + 1) + (m & 1)] : lin_r[2 * (pos - (kW - kH)) + (m & 1)];
    }
  };
  double acc = 0.0;
  int cur = 0;
  int d;
  bool given;
  if (hl == 0) {
    lam[cur][x + 1] = gT[gidx];  // lambda_T
    d = kH;
    given = true;
  } else {
    incoming(lam[cur], 2 * kH);
    d = 2 * kH - 1;
    given = false;
  }
  __syncthreads();
  const int dmin = hv > 0 ? 1 : kH;
  for (; d >= dmin; --d) {
    int at = cur;
    if (!given) {
      at = cur ^ 1;
      if (in_row(x, d)) lam[at][x + 1] = heat_update(lam[cur][x], lam[cur][x + 1], lam[cur][x + 2], k);
      __syncthreads();
    }
    given = false;
    const bool computed = !(hv == 0 && d == kH);
    if (computed && in_row(x, d)) {
      const double* u = hist[d - 1];
      const double lap = (u[x] + u[x + 2]) - 2.0 * u[x + 1];
      acc += lam[at][x + 1] * lap;
    }
    if (hv > 0 && d <= kH) {
      // two outermost values on each side of gap(d) go to the previous phase
      if (x == kA - d || x == kA - d + 1) lam_slots[base + sL + 2 * x + (d & 1)] = lam[at][x + 1];
      if (x == kA + d - 2 || x == kA + d - 1) lam_slots[base + sR + 2 * (x - kA + 1) + (d & 1)] = lam[at][x + 1];
    }
    if (hv == 0 && d == kH) g_ur[gidx] = lam[at][x + 1];
    if (d > kH && hl > 0) incoming(lam[at], d);
    __syncthreads();
    cur = at;
  }
  // per-tile sum in a fixed order, added to this tile's running sum
  red[x] = acc;
  __syncthreads();
  for (int s = kW / 2; s > 0; s >>= 1) {
    if (x < s) red[x] += red[x + s];
    __syncthreads();
  }
  if (x == 0) partial[b * nt + j] += red[0];
#undef ROW
}

__global__ void __launch_bounds__(kRemThreads)
rem_forward_kernel(const double* __restrict__ um, double* __restrict__ un, const Consts<double>* __restrict__ kb,
                   int64_t n, int batch) {
  const int64_t i = (int64_t)blockIdx.x * kRemThreads + threadIdx.x;
  if (i >= n * batch) return;
  const int64_t b = i / n, x = i % n;
  const double* v = um + b * n;
  const int64_t l = x == 0 ? n - 1 : x - 1;
  const int64_t r = x == n - 1 ? 0 : x + 1;
  un[i] = heat_update(v[l], v[x], v[r], kb[b]);
}

// lambda_m = A lambda_{m+1} and the dJ/dalpha term <lambda_{m+1}, L u_m>
// summed per block (fixed order), added to that block's running sum.
__global__ void __launch_bounds__(kRemThreads)
rem_adjoint_kernel(const double* __restrict__ lin, double* __restrict__ lout, const double* __restrict__ um,
                   double* __restrict__ partial, const Consts<double>* __restrict__ kb, int64_t n, int64_t nblk) {
  __shared__ double red[kRemThreads];
  const int64_t b = blockIdx.x / nblk;
  const int64_t x = (blockIdx.x % nblk) * kRemThreads + threadIdx.x;
  double acc = 0.0;
  if (x < n) {
    const double* l = lin + b * n;
    const double* u = um + b * n;
    const int64_t xl = x == 0 ? n - 1 : x - 1;
    const int64_t xr = x == n - 1 ? 0 : x + 1;
    lout[b * n + x] = heat_update(l[xl], l[x], l[xr], kb[b]);
    acc = l[x] * ((u[xl] + u[xr]) - 2.0 * u[x]);
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = kRemThreads / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] += red[0];
}

// g_alpha[b] = dt/dx^2 * (tile sums + remainder block sums), fixed order.
__global__ void __launch_bounds__(256)
reduce_kernel(const double* __restrict__ tiles, int64_t nt, const double* __restrict__ rem, int64_t nblk,
              double dfo, double* __restrict__ g_alpha) {
  __shared__ double red[256];
  const int64_t b = blockIdx.x;
  double acc = 0.0;
  for (int64_t i = threadIdx.x; i < nt; i += 256) acc += tiles[b * nt + i];
  for (int64_t i = threadIdx.x; i < nblk; i += 256) acc += rem[b * nblk + i];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) g_alpha[b] = dfo * red[0];
}

__global__ void fill_kernel(double* __restrict__ p, int64_t count) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = 0.0;
}

}  // namespace adj
}  // namespace swept

struct swept_adjoint_s {
  int32_t batch = 0;
  int64_t n = 0, steps = 0, nt = 0, nblk = 0;
  int K = 0;  // full phases of 32 steps; phases 0..K
  int r = 0;  // leading classic steps
  double dt = 0, dx = 0;
  int device = 0;
  bool have_forward = false;
  double* consts = nullptr;   // Consts<double>[batch]
  double* ckpt = nullptr;     // K phases x batch x 2nt x 66
  double* lam_slots = nullptr;
  double* rem = nullptr;      // (r+1) states x batch x n: u_0 .. u_r
  double* lam_a = nullptr;    // batch x n
  double* lam_b = nullptr;
  double* tiles = nullptr;    // batch x nt
  double* rparts = nullptr;   // batch x nblk
  size_t ckpt_bytes = 0;
};

namespace {

using swept::adj::kSL;
using swept::adj::kW;

int afail(int code, const std::string& m) { return swept::set_error(code, m); }
int ahip(hipError_t e, const char* what) { return afail(SWEPT_EDEVICE, std::string(what) + ": " + hipGetErrorString(e)); }

void adj_free(swept_adjoint_s* a) {
  for (double* q : {a->consts, a->ckpt, a->lam_slots, a->rem, a->lam_a, a->lam_b, a->tiles, a->rparts})
    if (q) (void)hipFree(q);
  delete a;
}

hipError_t zero(double* p, int64_t count, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(swept::adj::fill_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, p, count);
  return hipGetLastError();
}

}  // namespace

extern "C" {

int swept_adjoint_create(swept_adjoint* out, int32_t batch, int64_t n, int dtype, double dt, double dx,
                         int64_t steps) {
  if (!out) return afail(SWEPT_EINVAL, "out must not be NULL");
  *out = nullptr;
  if (batch < 1) return afail(SWEPT_EINVAL, "batch must be >= 1");
  if (dtype != SWEPT_F64) return afail(SWEPT_EUNSUPPORTED, "the adjoint is built for SWEPT_F64");
  if (n < kW || n % kW != 0) return afail(SWEPT_EUNSUPPORTED, "n must be a positive multiple of 64");
  if (steps < 1) return afail(SWEPT_EINVAL, "steps must be >= 1");
  if (!std::isfinite(dt) || !std::isfinite(dx) || dx == 0.0) return afail(SWEPT_EINVAL, "dt, dx must be finite, dx != 0");
  auto* a = new (std::nothrow) swept_adjoint_s();
  if (!a) return afail(SWEPT_ENOMEM, "host allocation failed");
  a->batch = batch;
  a->n = n;
  a->steps = steps;
  a->dt = dt;
  a->dx = dx;
  a->nt = n / kW;
  a->nblk = (n + swept::adj::kRemThreads - 1) / swept::adj::kRemThreads;
  a->r = (int)(steps % swept::adj::kH);
  a->K = (int)(steps / swept::adj::kH);
  hipError_t e = hipGetDevice(&a->device);
  if (e != hipSuccess) {
    delete a;
    return ahip(e, "hipGetDevice");
  }
  const size_t state = (size_t)batch * (size_t)n * sizeof(double);
  const size_t slots = (size_t)batch * 2 * (size_t)a->nt * kSL * sizeof(double);
  a->ckpt_bytes = (size_t)a->K * slots;
  struct Alloc {
    double** p;
    size_t bytes;
  } allocs[] = {
      {&a->consts, (size_t)batch * sizeof(swept::Consts<double>)},
      {&a->ckpt, std::max<size_t>(a->ckpt_bytes, 8)},
      {&a->lam_slots, slots},
      {&a->rem, (size_t)(a->r + 1) * state},
      {&a->lam_a, state},
      {&a->lam_b, state},
      {&a->tiles, (size_t)batch * (size_t)a->nt * sizeof(double)},
      {&a->rparts, (size_t)batch * (size_t)a->nblk * sizeof(double)},
  };
  for (const Alloc& al : allocs) {
    e = hipMalloc(reinterpret_cast<void**>(al.p), al.bytes);
    if (e != hipSuccess) {
      adj_free(a);
      return afail(SWEPT_ENOMEM, std::string("hipMalloc(adjoint workspace): ") + hipGetErrorString(e));
    }
  }
  *out = a;
  return SWEPT_OK;
}

int swept_forward_ckpt(swept_adjoint a, const void* u0, const double* alpha, void* uT, void* stream) {
  if (!a) return afail(SWEPT_EINVAL, "adjoint plan must not be NULL");
  if (!u0 || !alpha || !uT) return afail(SWEPT_EINVAL, "u0, alpha and uT must not be NULL");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int64_t total = (int64_t)a->batch * a->n;
  const size_t state = (size_t)total * sizeof(double);
  auto* k = reinterpret_cast<swept::Consts<double>*>(a->consts);
  hipLaunchKernelGGL(swept::adj::consts_kernel, dim3((unsigned)((a->batch + 63) / 64)), dim3(64), 0, st, alpha,
                     a->batch, a->dt, a->dx, k);
  hipError_t e = hipGetLastError();
  // leading classic steps: u_0 .. u_r kept for the reverse sweep
  if (e == hipSuccess) e = hipMemcpyAsync(a->rem, u0, state, hipMemcpyDeviceToDevice, st);
  for (int m = 0; m < a->r && e == hipSuccess; ++m) {
    hipLaunchKernelGGL(swept::adj::rem_forward_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st,
                       a->rem + (size_t)m * total, a->rem + (size_t)(m + 1) * total, k, a->n, a->batch);
    e = hipGetLastError();
  }
  const double* ur = a->rem + (size_t)a->r * total;
  const size_t pslots = (size_t)a->batch * 2 * (size_t)a->nt * kSL;
  if (a->K == 0) {
    if (e == hipSuccess) e = hipMemcpyAsync(uT, ur, state, hipMemcpyDeviceToDevice, st);
  } else {
    for (int p = 0; p <= a->K && e == hipSuccess; ++p) {
      const double* ck_in = p > 0 ? a->ckpt + (size_t)(p - 1) * pslots : nullptr;
      double* ck_out = p < a->K ? a->ckpt + (size_t)p * pslots : nullptr;
      hipLaunchKernelGGL(swept::adj::region_kernel<0>, dim3((unsigned)(a->batch * a->nt)), dim3(kW), 0, st, ur,
                         static_cast<double*>(uT), ck_in, ck_out, nullptr, nullptr, nullptr, nullptr, k, a->n, a->nt,
                         p, a->K);
      e = hipGetLastError();
    }
  }
  if (e != hipSuccess) return ahip(e, "swept_forward_ckpt");
  a->have_forward = true;
  return SWEPT_OK;
}

int swept_adjoint_run(swept_adjoint a, const void* g_uT, void* g_u0, double* g_alpha, void* stream) {
  if (!a) return afail(SWEPT_EINVAL, "adjoint plan must not be NULL");
  if (!g_uT || !g_u0 || !g_alpha) return afail(SWEPT_EINVAL, "g_uT, g_u0 and g_alpha must not be NULL");
  if (!a->have_forward) return afail(SWEPT_EINVAL, "swept_forward_ckpt must run first");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int64_t total = (int64_t)a->batch * a->n;
  const size_t state = (size_t)total * sizeof(double);
  auto* k = reinterpret_cast<const swept::Consts<double>*>(a->consts);
  const size_t pslots = (size_t)a->batch * 2 * (size_t)a->nt * kSL;
  hipError_t e = zero(a->tiles, (int64_t)a->batch * a->nt, st);
  if (e == hipSuccess) e = zero(a->rparts, (int64_t)a->batch * a->nblk, st);
  // lambda at tier r: from the swept sweep (or g_uT itself when T < 32)
  double* lam_r = a->r > 0 ? a->lam_a : static_cast<double*>(g_u0);
  if (a->K == 0) {
    if (e == hipSuccess) e = hipMemcpyAsync(lam_r, g_uT, state, hipMemcpyDeviceToDevice, st);
  } else {
    const double* ur = a->rem + (size_t)a->r * total;
    for (int p = a->K; p >= 0 && e == hipSuccess; --p) {
      const double* ck_in = p > 0 ? a->ckpt + (size_t)(p - 1) * pslots : nullptr;
      hipLaunchKernelGGL(swept::adj::region_kernel<1>, dim3((unsigned)(a->batch * a->nt)), dim3(kW), 0, st, ur,
                         nullptr, ck_in, nullptr, static_cast<const double*>(g_uT), a->lam_slots, lam_r, a->tiles, k,
                         a->n, a->nt, p, a->K);
      e = hipGetLastError();
    }
  }
  // leading classic steps backwards: lambda_m = A lambda_{m+1}, m = r-1 .. 0
  double* lin = lam_r;
  for (int m = a->r - 1; m >= 0 && e == hipSuccess; --m) {
    double* lout = m == 0 ? static_cast<double*>(g_u0) : (lin == a->lam_a ? a->lam_b : a->lam_a);
    hipLaunchKernelGGL(swept::adj::rem_adjoint_kernel, dim3((unsigned)(a->batch * a->nblk)),
                       dim3(swept::adj::kRemThreads), 0, st, lin, lout, a->rem + (size_t)m * total, a->rparts, k,
                       a->n, a->nblk);
    e = hipGetLastError();
    lin = lout;
  }
  if (e == hipSuccess) {
    hipLaunchKernelGGL(swept::adj::reduce_kernel, dim3((unsigned)a->batch), dim3(256), 0, st, a->tiles, a->nt,
                       a->rparts, a->nblk, a->dt / (a->dx * a->dx), g_alpha);
    e = hipGetLastError();
  }
  if (e != hipSuccess) return ahip(e, "swept_adjoint_run");
  return SWEPT_OK;
}

int swept_adjoint_info(swept_adjoint a, size_t* checkpoint_bytes, int* tile_width, int* steps_per_cycle,
                       int64_t* leading_classic_steps) {
  if (!a) return afail(SWEPT_EINVAL, "adjoint plan must not be NULL");
  if (checkpoint_bytes) *checkpoint_bytes = a->ckpt_bytes;
  if (tile_width) *tile_width = kW;
  if (steps_per_cycle) *steps_per_cycle = swept::adj::kH;
  if (leading_classic_steps) *leading_classic_steps = a->r;
  return SWEPT_OK;
}

void swept_adjoint_destroy(swept_adjoint a) {
  if (!a) return;
  adj_free(a);
}

}  // extern "C"
