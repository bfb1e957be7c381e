// Batched swept runs: thousands of independent periodic grids of uneven size,
// launched as one captured HIP graph.  The grids above the register-resident
// limit (all of them with the COMPACT or WAVE engine) are advanced by one
// persistent kernel of swept tiles; the smaller ones, with the default
// engine, run whole in register-resident kernels (resident_kernel below) on
// parallel branches of the same graph.
//
// Scheduling.  The grid of the persistent kernel is what the device holds
// resident (occupancy x CUs).  Each workgroup takes the next problem from a
// device-side counter -- problems are queued largest first, so the longest
// jobs start early and the tail is short -- and runs all swept phases of that
// problem itself: its NW waves share the problem's tiles within a phase and
// meet at a workgroup barrier between phases.  No workgroup ever waits for
// another, so every wave reaches the exit when the queue runs dry.
//
// Tiling of one problem of n points, split into 2 nt halves (nt tiles per
// tiling).  Even tile j is halves (2j, 2j+1), odd tile j is halves (2j+1,
// 2j+2 mod 2nt): the zig-zag of Sec. 4.2 with uneven tiles.  The phase height
// is the pure-triangle height of the smallest half (even for KS); larger
// halves carry a flat top.  The per-tile algorithm is either
//  - the compacted one (compact_tile.h, uneven-tile form, with LDS band
//    buffers and staging rows of its own for every wave): any n >= 32, halves
//    measured in points (compact::uneven_tiling: all but the last a multiple
//    of 4 s, every one at most 32 P points); or
//  - the register engine's (wave_tile.h), whose halves are whole lanes: n a
//    multiple of P, c = n/P lane-chunks, halves of floor(c/2nt) or
//    ceil(c/2nt) lanes with nt = ceil(c/64).
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <numeric>
#include <string>
#include <vector>

#include "compact_tile.h"
#include "internal.h"
#include "poison.h"
#include "swept.h"
#include "wave_tile.h"

namespace swept {
namespace {

constexpr int kBatchNW = 4;  // waves per workgroup

template <typename T>
struct BatchItem {
  int64_t u_off;     // first point of this ring in the concatenated state
  int64_t slot_off;  // first value of its 2 nt edge slots
  int32_t n;         // ring points
  int32_t nt;        // tiles per tiling
  int32_t h;         // tiers per full phase
  int32_t pad;
  Consts<T> k;
};

__global__ void batch_reset_kernel(int* queue) { *queue = 0; }

// COMPACT: 0 register engine, 1 compacted engine.
template <int KIND, typename T, int P, int NW, int COMPACT>
__global__ void __launch_bounds__(64 * NW)
batch_kernel(const BatchItem<T>* __restrict__ items, int nitems, T* u, T* slots, int64_t tiers, int* queue,
             int poison) {
  constexpr int S = Radius<KIND>::value;
  constexpr int SLEN = 64 * P + 2 * S;
  constexpr int NB = COMPACT ? compact::Lds<KIND, P>::band : 1;
  constexpr int NS = COMPACT ? compact::Lds<KIND, P>::stage : 1;
  __shared__ T sbm[NW][NB];   // per wave: edge bands of the tile in hand
  __shared__ T stgm[NW][NS];  // per wave: staging row for layout changes
  __shared__ int s_item;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  for (;;) {
    if (threadIdx.x == 0) s_item = atomicAdd(queue, 1);
    __syncthreads();
    const int it = s_item;
    __syncthreads();  // every wave has read s_item before it is overwritten
    if (it >= nitems) break;
    const BatchItem<T> pr = items[it];
    T* ring = u + pr.u_off;
    T* slotA = slots + pr.slot_off;
    T* slotB = slotA + (int64_t)pr.nt * SLEN;
    const int halves = 2 * pr.nt;
    const int c = pr.n / P;  // register engine: lanes of P points
    const int hb = c / halves;
    const int hx = c % halves;
    const compact::Uneven ut = compact::uneven_tiling(pr.n, P, S);  // compacted engine: halves in points
    const int64_t full = tiers / pr.h;
    const int rem = (int)(tiers % pr.h);
    const int64_t ne = full + (rem ? 1 : 0);  // edge sets; phases = ne + 1
    for (int64_t ph = 0; ph <= ne; ++ph) {
      const int hv = ph == 0 ? 0 : (ph - 1 < full ? pr.h : rem);
      const int hl = ph == ne ? 0 : (ph < full ? pr.h : rem);
      const int parity = (int)(ph & 1);
      for (int j = wave; j < pr.nt; j += NW) {
        const int iL = 2 * j + parity;
        const int iR = (iL + 1) % halves;
        T* sL = parity ? slotB + (int64_t)j * SLEN : slotA + (int64_t)j * SLEN;
        T* sR = parity ? slotA + (int64_t)((j + 1) % pr.nt) * SLEN : slotB + (int64_t)j * SLEN;
        if constexpr (COMPACT) {
          if (poison) {
            // this tile's use of the wave's LDS starts from NaN
            poison_lds(sbm[wave], NB, lane, 64);
            poison_lds(stgm[wave], NS, lane, 64);
            compact::wave_sync();
          }
          compact::tile_phase_g<KIND, T, P>(ring, pr.n, compact::uneven_origin(ut, iL), sL, sR,
                                            compact::uneven_width(ut, iL), compact::uneven_width(ut, iR), hv, hl,
                                            pr.k, lane, sbm[wave], stgm[wave]);
        } else {
          wave::Tile<T> g;
          g.origin = (int64_t)(iL * hb + min(iL, hx)) * P;
          g.kL = hb + (iL < hx ? 1 : 0);
          g.kR = hb + (iR < hx ? 1 : 0);
          g.sL = sL;
          g.sR = sR;
          wave::tile_phase<KIND, T, P, 3>(ring, pr.n, g, hv, hl, pr.k, lane);
        }
      }
      // the next phase's tiles read slots other waves of this group wrote
      __threadfence();
      __syncthreads();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
  }
}

// Whole-grid kernel for the grids that fit one workgroup's registers
// (n <= kResMax): one workgroup per grid, lane g of its NW waves holding
// points [16 g, 16 g + 16) of the ring for all the steps.  Grids come in
// four classes by size, each with its own workgroup size (1, 4, 8 or 16
// waves), so a small grid does not hold a whole CU's registers.  A grid this small
// needs no decomposition in time: every sub-step updates every point, so no
// lane idles on a triangle and no edge band is selected or stored; only the
// halos move -- by lane shifts inside a wave, and through a small LDS
// exchange (double-buffered by sub-step parity, one workgroup barrier per
// sub-step) between waves and across the periodic seam.  Each point gets the
// same update in the same order as in every other engine, so the results are
// the naive run's bit for bit.
//
// Any n: the ring's c = ceil(n/16) lanes hold 16 points each but the last,
// which holds M = n - 16 (c - 1) (1 .. 16).  M is a compile-time case of the
// kernel.  At each exchange the last lane writes the ring's first two points
// (its right halo) into its registers M and M + 1 -- for M = 15 the second goes
// to its right halo value -- so its valid points read them in place, and the
// lane to its left, which reads the last lane's first two registers, sees
// point 0 where the last lane ends after one point (M = 1).  The points in its
// registers above M + 1 are don't-care.  The ring's last two points (the left
// halo of lane 0) come from registers M - 2 and M - 1 of the last lane, or,
// for M = 1, from the last register of the lane before it.
constexpr int kResQ = 16;                // points per lane
constexpr int kResClasses = 4;
constexpr int kResWaves[kResClasses] = {16, 8, 4, 1};  // waves per workgroup of each size class
constexpr int kResMax = kResQ * 64 * 16;  // 16384 points

// Size class of a resident grid: the smallest workgroup that holds it.
__host__ __device__ constexpr int res_class(int64_t n) {
  return n > kResQ * 64 * 8 ? 0 : (n > kResQ * 64 * 4 ? 1 : (n > kResQ * 64 ? 2 : 3));
}
// Side stream of each size class: the two small classes share one, so the
// persistent kernel's stream and the side streams fit four hardware queues.
constexpr int kResStreams = 3;
constexpr int kResStreamOf[kResClasses] = {0, 1, 2, 2};

// LDS halo exchange buffers of one resident workgroup.
template <typename T, int NW, int D>
struct ResLds {
  T edF[2][NW][D];  // per wave: the first D points of its lane 0
  T edL[2][NW][D];  // per wave: the last D points of its lane 63
  T edC[2][D];      // the last D points of the ring
};

template <int KIND, typename T, int NW, int M>
__device__ __forceinline__ void resident_body(const BatchItem<T>& pr, T* u, int64_t steps, ResLds<T, NW, 2>& L) {
  static_assert(Radius<KIND>::value <= 2, "one exchange holds two halo points per side");
  static_assert(M >= 1 && M <= kResQ, "points in the last lane");
  constexpr int Q = kResQ;
  // halo depth of one exchange: two points per side, which is one KS
  // sub-step or two heat steps
  constexpr int D = 2;
  const int g = threadIdx.x;
  const int lane = g & 63;
  const int wv = g >> 6;
  const int c = (pr.n + Q - 1) / Q;   // lanes holding points
  const bool busy = wv * 64 < c;      // wave-uniform: the wave holds points
  const bool active = g < c;
  const bool rag = g == c - 1;        // the ring's last lane (M points)
  // halos that do not come from the neighbouring lane of the same wave
  const bool first = active && lane == 0;
  const bool last = active && (lane == 63 || rag);
  T* ring = u + pr.u_off;
  T A[Q], B[Q];
#pragma unroll
  for (int i = 0; i < Q; ++i) A[i] = (active && (i < M || !rag)) ? ring[(int64_t)g * Q + i] : T(0);
  int sub = 0;
  // Publish this lane's edge points, then gather the D halo points per side
  // of src: lo[i] = point i - D, hi[i] = point Q + i.  The last lane first
  // takes the ring's first points into its registers M, M + 1.
  auto exchange = [&](T (&src)[Q], T (&lo)[D], T (&hi)[D]) {
    const int bf = sub & 1;
    if (busy) {
      if (active && lane == 0)
#pragma unroll
        for (int i = 0; i < D; ++i) L.edF[bf][wv][i] = src[i];
      if (active && lane == 63)
#pragma unroll
        for (int i = 0; i < D; ++i) L.edL[bf][wv][i] = src[Q - D + i];
      if (rag) {
#pragma unroll
        for (int i = 0; i < D; ++i)
          if (M - D + i >= 0) L.edC[bf][i] = src[M - D + i];
      }
      if constexpr (M < D) {
        if (g == c - 2)
#pragma unroll
          for (int i = 0; i < D - M; ++i) L.edC[bf][i] = src[Q - (D - M) + i];
      }
    }
    __syncthreads();
    T xl[D] = {}, xr[D] = {};
    if (first) {
#pragma unroll
      for (int i = 0; i < D; ++i) xl[i] = g == 0 ? L.edC[bf][i] : L.edL[bf][wv - 1][i];
    }
    if (last) {
#pragma unroll
      for (int i = 0; i < D; ++i) xr[i] = rag ? L.edF[bf][0][i] : L.edF[bf][wv + 1][i];
    }
    if constexpr (M < Q) {
      src[M] = wave::pick(rag, xr[0], src[M]);
      if constexpr (M + 1 < Q) src[M + 1] = wave::pick(rag, xr[1], src[M + 1]);
    }
    wave::halos<T, Q, D, true>(src, xl, xr, first, last, lo, hi);
    if constexpr (M == Q - 1) hi[0] = wave::pick(rag, xr[1], hi[0]);
    if constexpr (M == 1) {
      // the lane before the last reads point 0 as its second right halo
      // point (also when it ends a wave, where edF holds the unpatched value)
      const T p0 = L.edF[bf][0][0];
      hi[1] = wave::pick(g == c - 2, p0, hi[1]);
    }
    ++sub;
  };
  const Consts<T> k = pr.k;
  if constexpr (KIND == kHeat) {
    // Two steps per exchange: the first step also forms points -1 and Q
    // (the neighbours' edge points, from the same three values in the same
    // order, so the same bits), the second uses them; A -> B -> A, so no
    // register moves back.
    for (int64_t s = 0; s + 1 < steps; s += 2) {
      T lo[D], hi[D];
      exchange(A, lo, hi);
      if (busy) {
        const T m1 = heat_update(lo[0], lo[1], A[0], k);          // point -1
        const T pq = heat_update(A[Q - 1], hi[0], hi[1], k);      // point Q
#pragma unroll
        for (int i = 0; i < Q; ++i)
          B[i] = heat_update(i > 0 ? A[i - 1] : lo[1], A[i], i + 1 < Q ? A[i + 1] : hi[0], k);
#pragma unroll
        for (int i = 0; i < Q; ++i)
          A[i] = heat_update(i > 0 ? B[i - 1] : m1, B[i], i + 1 < Q ? B[i + 1] : pq, k);
      }
    }
    if (steps & 1) {
      T lo[D], hi[D];
      exchange(A, lo, hi);
      if (busy) {
#pragma unroll
        for (int i = 0; i < Q; ++i)
          B[i] = heat_update(i > 0 ? A[i - 1] : lo[1], A[i], i + 1 < Q ? A[i + 1] : hi[0], k);
#pragma unroll
        for (int i = 0; i < Q; ++i) A[i] = B[i];
      }
    }
  } else {
    for (int64_t s = 0; s < steps; ++s) {
      T lo[D], hi[D];
      exchange(A, lo, hi);
      if (busy) {
#pragma unroll
        for (int i = 0; i < Q; ++i)
          B[i] = ks_predictor(wave::at<T, Q, D>(A, lo, hi, i - 2), wave::at<T, Q, D>(A, lo, hi, i - 1), A[i],
                              wave::at<T, Q, D>(A, lo, hi, i + 1), wave::at<T, Q, D>(A, lo, hi, i + 2), k);
      }
      exchange(B, lo, hi);
      if (busy) {
#pragma unroll
        for (int i = 0; i < Q; ++i)
          A[i] = ks_final(A[i], wave::at<T, Q, D>(B, lo, hi, i - 2), wave::at<T, Q, D>(B, lo, hi, i - 1), B[i],
                          wave::at<T, Q, D>(B, lo, hi, i + 1), wave::at<T, Q, D>(B, lo, hi, i + 2), k);
      }
    }
  }
  if (active) {
#pragma unroll
    for (int i = 0; i < Q; ++i)
      if (i < M || !rag) ring[(int64_t)g * Q + i] = A[i];
  }
}

template <int KIND, typename T, int NW>
__global__ void __launch_bounds__(64 * NW)
resident_kernel(const BatchItem<T>* __restrict__ items, T* u, int64_t steps, int poison) {
  __shared__ ResLds<T, NW, 2> L;
  if (poison) {
    poison_lds(reinterpret_cast<T*>(&L), (int)(sizeof(L) / sizeof(T)), (int)threadIdx.x, 64 * NW);
    __syncthreads();
  }
  const BatchItem<T> pr = items[blockIdx.x];
  // points in the ring's last lane (workgroup-uniform)
  switch (pr.n - (pr.n - 1) / kResQ * kResQ) {
    case 1: resident_body<KIND, T, NW, 1>(pr, u, steps, L); break;
    case 2: resident_body<KIND, T, NW, 2>(pr, u, steps, L); break;
    case 3: resident_body<KIND, T, NW, 3>(pr, u, steps, L); break;
    case 4: resident_body<KIND, T, NW, 4>(pr, u, steps, L); break;
    case 5: resident_body<KIND, T, NW, 5>(pr, u, steps, L); break;
    case 6: resident_body<KIND, T, NW, 6>(pr, u, steps, L); break;
    case 7: resident_body<KIND, T, NW, 7>(pr, u, steps, L); break;
    case 8: resident_body<KIND, T, NW, 8>(pr, u, steps, L); break;
    case 9: resident_body<KIND, T, NW, 9>(pr, u, steps, L); break;
    case 10: resident_body<KIND, T, NW, 10>(pr, u, steps, L); break;
    case 11: resident_body<KIND, T, NW, 11>(pr, u, steps, L); break;
    case 12: resident_body<KIND, T, NW, 12>(pr, u, steps, L); break;
    case 13: resident_body<KIND, T, NW, 13>(pr, u, steps, L); break;
    case 14: resident_body<KIND, T, NW, 14>(pr, u, steps, L); break;
    case 15: resident_body<KIND, T, NW, 15>(pr, u, steps, L); break;
    default: resident_body<KIND, T, NW, 16>(pr, u, steps, L); break;
  }
}

}  // namespace
}  // namespace swept

using swept::BatchItem;
using swept::Consts;

namespace {
int bfail(int code, const std::string& m) { return swept::set_error(code, m); }
int bhip(hipError_t e, const char* what) { return bfail(SWEPT_EDEVICE, std::string(what) + ": " + hipGetErrorString(e)); }
}  // namespace

struct swept_batch_s {
  int kind = 0, dtype = 0;
  int32_t nprob = 0;
  int64_t steps = 0;
  int64_t total_points = 0;
  std::vector<int64_t> offsets;  // per problem, input order
  // host copy of the problems, to rebuild the tiling when the engine changes
  std::vector<int64_t> n;
  std::vector<double> dt, dx, alpha;
  std::vector<int32_t> order;  // queue order: largest first
  int P = 16;                  // points per lane of the current tiling
  int32_t nswept = 0;          // grids run by the persistent swept kernel
  int32_t nres = 0;            // grids run whole by the resident kernels (AUTO engine)
  int32_t res_count[swept::kResClasses] = {};  // resident grids per size class (16, 8, 4, 1 waves)
  void* items = nullptr;       // device BatchItem<T>[nswept], queue order
  void* res_items = nullptr;   // device BatchItem<T>[nres], largest first (so by class)
  void* slots = nullptr;
  size_t slots_bytes = 0;
  int* queue = nullptr;
  int device = 0;
  int engine = SWEPT_ENGINE_AUTO;
  bool poison = false;             // SWEPT_DEBUG_POISON: NaN-fill the slots (and LDS) before each run
  int checks = 0;                  // SWEPT_CHECK_* flags (swept_batch_set_checks)
  int* flag = nullptr;             // device flag of the non-finite check
  int grid = 0;
  hipStream_t cap_stream = nullptr;
  hipStream_t side[swept::kResStreams] = {};  // branches of the resident classes, beside the persistent kernel
  hipEvent_t ev_fork = nullptr;
  hipEvent_t ev_join[swept::kResStreams] = {};
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  void* graph_u = nullptr;
};

namespace {

bool compact_engine(int engine) { return engine != SWEPT_ENGINE_WAVE; }

// Points per lane of the swept tiling an engine runs.  With every grid in
// the persistent kernel (COMPACT), heat takes 8: half the LDS and registers
// per wave, so three workgroups share a CU and the many small grids keep it
// busy (measured on the 4096-grid workload: 3.84e12 at 8 vs 3.17e12 at 16
// cell-updates/s).  Everything else takes 16 -- with AUTO and RESIDENT the
// small grids run in the resident kernels, and the large ones gain from the
// wider tiles (grids above 16384 points: 3.82e12 at 16 vs 3.03e12 at 8);
// KS 5.02e11 at 16 vs 4.75e11 at 8; register heat 3.02e12 at 16 vs 2.70e12
// at 8.
int points_per_lane(int kind, int engine) { return engine == SWEPT_ENGINE_COMPACT && kind == SWEPT_HEAT_FTCS ? 8 : 16; }

template <int KIND, typename T, int P, int C>
void* batch_kernel_ptr() {
  return reinterpret_cast<void*>(swept::batch_kernel<KIND, T, P, swept::kBatchNW, C>);
}

template <int P, int C>
void* kernel_for_pc(int kind, int dtype) {
  if (kind == SWEPT_HEAT_FTCS)
    return dtype == SWEPT_F64 ? batch_kernel_ptr<swept::kHeat, double, P, C>()
                              : batch_kernel_ptr<swept::kHeat, float, P, C>();
  return dtype == SWEPT_F64 ? batch_kernel_ptr<swept::kKS, double, P, C>() : batch_kernel_ptr<swept::kKS, float, P, C>();
}

void* kernel_for(const swept_batch_s* b) {
  const bool c = compact_engine(b->engine);
  if (b->P == 8) return c ? kernel_for_pc<8, 1>(b->kind, b->dtype) : kernel_for_pc<8, 0>(b->kind, b->dtype);
  return c ? kernel_for_pc<16, 1>(b->kind, b->dtype) : kernel_for_pc<16, 0>(b->kind, b->dtype);
}

template <int KIND, typename T, int P, int C>
void launch_batch(const swept_batch_s* b, void* u, int64_t tiers, hipStream_t st) {
  hipLaunchKernelGGL((swept::batch_kernel<KIND, T, P, swept::kBatchNW, C>), dim3((unsigned)b->grid),
                     dim3(64 * swept::kBatchNW), 0, st, static_cast<const BatchItem<T>*>(b->items), b->nswept,
                     static_cast<T*>(u), static_cast<T*>(b->slots), tiers, b->queue, (int)b->poison);
}

// Launch the resident grids of size class cl (0: 16 waves, 1: 8, 2: 4, 3: 1).
template <int KIND, typename T>
void launch_resident(const swept_batch_s* b, int cl, void* u, hipStream_t st) {
  const auto* items = static_cast<const BatchItem<T>*>(b->res_items);
  int32_t first = 0;
  for (int c = 0; c < cl; ++c) first += b->res_count[c];
  const int32_t cnt = b->res_count[cl];
  if (cnt <= 0) return;
  const dim3 grid((unsigned)cnt), block((unsigned)(64 * swept::kResWaves[cl]));
  if (cl == 0)
    hipLaunchKernelGGL((swept::resident_kernel<KIND, T, swept::kResWaves[0]>), grid, block, 0, st, items + first,
                       static_cast<T*>(u), b->steps,
                       (int)b->poison);
  else if (cl == 1)
    hipLaunchKernelGGL((swept::resident_kernel<KIND, T, swept::kResWaves[1]>), grid, block, 0, st, items + first,
                       static_cast<T*>(u), b->steps,
                       (int)b->poison);
  else if (cl == 2)
    hipLaunchKernelGGL((swept::resident_kernel<KIND, T, swept::kResWaves[2]>), grid, block, 0, st, items + first,
                       static_cast<T*>(u), b->steps,
                       (int)b->poison);
  else
    hipLaunchKernelGGL((swept::resident_kernel<KIND, T, swept::kResWaves[3]>), grid, block, 0, st, items + first,
                       static_cast<T*>(u), b->steps,
                       (int)b->poison);
}

template <int P, int C>
void launch_batch_pc(const swept_batch_s* b, void* u, int64_t tiers, hipStream_t st) {
  if (b->kind == SWEPT_HEAT_FTCS) {
    if (b->dtype == SWEPT_F64)
      launch_batch<swept::kHeat, double, P, C>(b, u, tiers, st);
    else
      launch_batch<swept::kHeat, float, P, C>(b, u, tiers, st);
  } else {
    if (b->dtype == SWEPT_F64)
      launch_batch<swept::kKS, double, P, C>(b, u, tiers, st);
    else
      launch_batch<swept::kKS, float, P, C>(b, u, tiers, st);
  }
}

hipError_t launch_resident_class(swept_batch_s* b, int cl, void* u, hipStream_t st) {
  if (b->kind == SWEPT_HEAT_FTCS) {
    if (b->dtype == SWEPT_F64)
      launch_resident<swept::kHeat, double>(b, cl, u, st);
    else
      launch_resident<swept::kHeat, float>(b, cl, u, st);
  } else {
    if (b->dtype == SWEPT_F64)
      launch_resident<swept::kKS, double>(b, cl, u, st);
    else
      launch_resident<swept::kKS, float>(b, cl, u, st);
  }
  return hipGetLastError();
}

// Streams and events of the side branches, made on first use.
hipError_t ensure_side(swept_batch_s* b) {
  hipError_t e = hipSuccess;
  if (!b->ev_fork) e = hipEventCreateWithFlags(&b->ev_fork, hipEventDisableTiming);
  for (int q = 0; q < swept::kResStreams && e == hipSuccess; ++q) {
    if (!b->side[q]) e = hipStreamCreateWithFlags(&b->side[q], hipStreamNonBlocking);
    if (e == hipSuccess && !b->ev_join[q]) e = hipEventCreateWithFlags(&b->ev_join[q], hipEventDisableTiming);
  }
  return e;
}

hipError_t launch_swept(swept_batch_s* b, void* u, hipStream_t st);

// The grids are independent, so the kernels run side by side: the resident
// size classes go on side streams (the two small ones sharing one), forked
// from and joined back to `st` by events (parallel branches of the captured
// graph), beside the persistent kernel on `st`.  Run one after another, the
// classes would end well after the persistent kernel (heat: 65.7 ms against
// 52.0 ms).
hipError_t enqueue_runs(swept_batch_s* b, void* u, hipStream_t st);

// The batch's launches, then (with the non-finite check on) the scan of every
// grid's values.
hipError_t enqueue_batch(swept_batch_s* b, void* u, hipStream_t st) {
  hipError_t e = enqueue_runs(b, u, st);
  if (e == hipSuccess && (b->checks & SWEPT_CHECK_NONFINITE))
    e = swept::enqueue_nonfinite_check(u, b->total_points, b->dtype == SWEPT_F64 ? 8 : 4, b->flag, st);
  return e;
}

hipError_t enqueue_runs(swept_batch_s* b, void* u, hipStream_t st) {
  if (b->nres == 0) return launch_swept(b, u, st);
  bool used[swept::kResStreams] = {};
  for (int cl = 0; cl < swept::kResClasses; ++cl)
    if (b->res_count[cl] > 0) used[swept::kResStreamOf[cl]] = true;
  hipError_t e = ensure_side(b);
  if (e == hipSuccess) e = hipEventRecord(b->ev_fork, st);
  for (int q = 0; q < swept::kResStreams && e == hipSuccess; ++q)
    if (used[q]) e = hipStreamWaitEvent(b->side[q], b->ev_fork, 0);
  for (int cl = 0; cl < swept::kResClasses && e == hipSuccess; ++cl)
    if (b->res_count[cl] > 0) e = launch_resident_class(b, cl, u, b->side[swept::kResStreamOf[cl]]);
  if (e == hipSuccess) e = launch_swept(b, u, st);
  for (int q = 0; q < swept::kResStreams && e == hipSuccess; ++q) {
    if (!used[q]) continue;
    e = hipEventRecord(b->ev_join[q], b->side[q]);
    if (e == hipSuccess) e = hipStreamWaitEvent(st, b->ev_join[q], 0);
  }
  return e;
}

hipError_t launch_swept(swept_batch_s* b, void* u, hipStream_t st) {
  if (b->nswept == 0) return hipSuccess;
  if (b->poison) {
    const hipError_t pe =
        swept::poison_fill(b->slots, b->slots_bytes, b->dtype == SWEPT_F64 ? 8 : 4, st);
    if (pe != hipSuccess) return pe;
  }
  hipLaunchKernelGGL(swept::batch_reset_kernel, dim3(1), dim3(1), 0, st, b->queue);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t tiers = b->steps * (b->kind == SWEPT_KS_RK2 ? 2 : 1);
  const bool c = compact_engine(b->engine);
  if (b->P == 8) {
    if (c)
      launch_batch_pc<8, 1>(b, u, tiers, st);
    else
      launch_batch_pc<8, 0>(b, u, tiers, st);
  } else {
    if (c)
      launch_batch_pc<16, 1>(b, u, tiers, st);
    else
      launch_batch_pc<16, 0>(b, u, tiers, st);
  }
  return hipGetLastError();
}

// Persistent grid: as many workgroups as the device holds at once.
hipError_t size_grid(swept_batch_s* b) {
  int per_cu = 0, cus = 0;
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel_for(b), 64 * swept::kBatchNW, 0);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, b->device);
  if (e != hipSuccess) return e;
  if (per_cu < 1) per_cu = 1;
  b->grid = (int)std::min<int64_t>((int64_t)per_cu * cus, b->nswept);
  return hipSuccess;
}

void drop_graph(swept_batch_s* b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
  b->graph_u = nullptr;
}

template <typename T>
Consts<T> consts_for(double dt, double dx, double alpha) {
  return swept::make_consts<T>(dt, dx, alpha);  // the host formulas of swept_plan_create (Sec. 4.1, Sec. 5)
}

// Largest grid an engine runs whole in the resident kernels (0: none): with
// AUTO and RESIDENT, every grid that fits one workgroup's registers.  Their
// workgroups run beside the persistent kernel, whose P = 16 workgroups (one
// per CU) leave room for them.  Measured on the 4096-grid heat workload:
// 63.7 ms, against 65.1 ms with only the 1- and 4-wave classes resident and
// 71.1 ms with every grid as P = 8 compacted tiles (which in turn beat the
// resident kernels beside P = 8 tiles, 70.7 against 75.9 ms: the 16-wave
// workgroups then waited for free CUs).  KS: 434 ms against 475 ms.
int64_t resident_max(int kind, int engine) {
  (void)kind;
  return engine == SWEPT_ENGINE_RESIDENT || engine == SWEPT_ENGINE_AUTO ? swept::kResMax : 0;
}

// Whether grid i runs whole in the resident kernels.
bool resident(const swept_batch_s* b, int engine, int32_t i) {
  return b->n[(size_t)i] <= resident_max(b->kind, engine);
}

// Descriptors of the resident grids (largest first; no slots).
template <typename T>
std::vector<BatchItem<T>> make_res_items(const swept_batch_s* b, int engine) {
  std::vector<BatchItem<T>> items;
  for (int32_t i : b->order) {
    if (!resident(b, engine, i)) continue;
    BatchItem<T> it{};
    it.u_off = b->offsets[(size_t)i];
    it.n = (int32_t)b->n[(size_t)i];
    it.k = consts_for<T>(b->dt[(size_t)i], b->dx[(size_t)i], b->kind == SWEPT_HEAT_FTCS ? b->alpha[(size_t)i] : 0.0);
    items.push_back(it);
  }
  return items;
}

// Grid descriptors of the swept grids' tiling with P points per lane, in
// queue order.
template <typename T>
std::vector<BatchItem<T>> make_items(const swept_batch_s* b, int engine, int P, size_t* slot_values) {
  const int S = b->kind == SWEPT_KS_RK2 ? 2 : 1;
  const int64_t slen = 64 * P + 2 * S;
  std::vector<BatchItem<T>> items;
  int64_t soff = 0;
  for (int32_t i : b->order) {
    if (resident(b, engine, i)) continue;
    items.emplace_back();
    BatchItem<T>& it = items.back();
    const int64_t n = b->n[(size_t)i];
    it.u_off = b->offsets[(size_t)i];
    it.slot_off = soff;
    it.n = (int32_t)n;
    int h;
    if (compact_engine(engine)) {
      // halves in points, at most 32 P each (compact::uneven_tiling)
      const swept::compact::Uneven ut = swept::compact::uneven_tiling(n, P, S);
      it.nt = (int32_t)ut.nt;
      h = swept::compact::uneven_full_tiers(ut, S);
    } else {
      // halves of whole lanes of P points (n a multiple of P)
      const int c = (int)(n / P);
      it.nt = (c + 63) / 64;
      h = c / (2 * it.nt) * P / S;
    }
    if (b->kind == SWEPT_KS_RK2) h &= ~1;
    it.h = h;
    it.pad = 0;
    it.k = consts_for<T>(b->dt[(size_t)i], b->dx[(size_t)i], b->kind == SWEPT_HEAT_FTCS ? b->alpha[(size_t)i] : 0.0);
    soff += 2 * (int64_t)it.nt * slen;
  }
  *slot_values = (size_t)soff;
  return items;
}

// Upload host bytes to a new device buffer (at least 8 bytes).
hipError_t upload(void** out, const void* host, size_t bytes) {
  *out = nullptr;
  hipError_t e = hipMalloc(out, std::max<size_t>(bytes, 8));
  if (e == hipSuccess && bytes) e = hipMemcpy(*out, host, bytes, hipMemcpyHostToDevice);
  if (e != hipSuccess && *out) {
    (void)hipFree(*out);
    *out = nullptr;
  }
  return e;
}

// (Re)build the device descriptors of both kernels and the edge slots of the
// swept grids for an engine and P points per lane.  On failure the plan
// keeps its previous tiling.
int build_tiling(swept_batch_s* b, int engine, int P) {
  int32_t count[swept::kResClasses] = {};
  for (int32_t i : b->order)
    if (resident(b, engine, i)) ++count[swept::res_class(b->n[(size_t)i])];
  // one launch per class, one workgroup per grid: its work-items must fit 32 bits
  for (int cl = 0; cl < swept::kResClasses; ++cl)
    if ((int64_t)count[cl] * 64 * swept::kResWaves[cl] > (int64_t)UINT32_MAX)
      return bfail(SWEPT_EUNSUPPORTED, "too many resident grids of one size class for one launch");
  size_t slot_values = 0, item_bytes = 0, res_bytes = 0;
  const void* host_items = nullptr;
  const void* host_res = nullptr;
  std::vector<BatchItem<double>> id, rd;
  std::vector<BatchItem<float>> ifl, rf;
  size_t nsw = 0, nre = 0;
  if (b->dtype == SWEPT_F64) {
    id = make_items<double>(b, engine, P, &slot_values);
    rd = make_res_items<double>(b, engine);
    host_items = id.data();
    host_res = rd.data();
    nsw = id.size();
    nre = rd.size();
    item_bytes = nsw * sizeof(BatchItem<double>);
    res_bytes = nre * sizeof(BatchItem<double>);
  } else {
    ifl = make_items<float>(b, engine, P, &slot_values);
    rf = make_res_items<float>(b, engine);
    host_items = ifl.data();
    host_res = rf.data();
    nsw = ifl.size();
    nre = rf.size();
    item_bytes = nsw * sizeof(BatchItem<float>);
    res_bytes = nre * sizeof(BatchItem<float>);
  }
  const size_t es = b->dtype == SWEPT_F64 ? sizeof(double) : sizeof(float);
  void* items = nullptr;
  void* res = nullptr;
  void* slots = nullptr;
  hipError_t e = upload(&items, host_items, item_bytes);
  if (e == hipSuccess) e = upload(&res, host_res, res_bytes);
  if (e == hipSuccess) e = hipMalloc(&slots, std::max<size_t>(slot_values * es, 8));
  if (e != hipSuccess) {
    if (items) (void)hipFree(items);
    if (res) (void)hipFree(res);
    return bfail(SWEPT_ENOMEM, std::string("hipMalloc/hipMemcpy(batch): ") + hipGetErrorString(e));
  }
  if (b->items) (void)hipFree(b->items);
  if (b->res_items) (void)hipFree(b->res_items);
  if (b->slots) (void)hipFree(b->slots);
  b->items = items;
  b->res_items = res;
  b->slots = slots;
  b->slots_bytes = slot_values * es;
  b->nswept = (int32_t)nsw;
  b->nres = (int32_t)nre;
  for (int cl = 0; cl < swept::kResClasses; ++cl) b->res_count[cl] = count[cl];
  b->P = P;
  return SWEPT_OK;
}

void batch_free(swept_batch_s* b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
  for (int q = 0; q < swept::kResStreams; ++q) {
    if (b->side[q]) (void)hipStreamDestroy(b->side[q]);
    if (b->ev_join[q]) (void)hipEventDestroy(b->ev_join[q]);
  }
  if (b->ev_fork) (void)hipEventDestroy(b->ev_fork);
  if (b->items) (void)hipFree(b->items);
  if (b->res_items) (void)hipFree(b->res_items);
  if (b->slots) (void)hipFree(b->slots);
  if (b->queue) (void)hipFree(b->queue);
  if (b->flag) (void)hipFree(b->flag);
  delete b;
}

}  // namespace

extern "C" {

int swept_batch_create(swept_batch* out, int32_t nprob, const int64_t* n, int kind, int dtype, const double* dt,
                       const double* dx, const double* alpha, int64_t steps) {
  if (!out) return bfail(SWEPT_EINVAL, "out must not be NULL");
  *out = nullptr;
  if (kind != SWEPT_HEAT_FTCS && kind != SWEPT_KS_RK2) return bfail(SWEPT_EINVAL, "unknown stencil kind");
  if (dtype != SWEPT_F32 && dtype != SWEPT_F64) return bfail(SWEPT_EINVAL, "unknown dtype");
  if (nprob < 1) return bfail(SWEPT_EINVAL, "nprob must be >= 1");
  if (!n || !dt || !dx || (kind == SWEPT_HEAT_FTCS && !alpha)) return bfail(SWEPT_EINVAL, "null host array");
  if (steps < 0) return bfail(SWEPT_EINVAL, "steps must be >= 0");
  for (int32_t i = 0; i < nprob; ++i) {
    if (n[i] < 32 || n[i] > (int64_t)1 << 30)
      return bfail(SWEPT_EUNSUPPORTED, "problem " + std::to_string(i) + ": n must be at least 32 and at most 2^30");
    if (!std::isfinite(dt[i]) || !std::isfinite(dx[i]) || dx[i] == 0.0 ||
        (kind == SWEPT_HEAT_FTCS && !std::isfinite(alpha[i])))
      return bfail(SWEPT_EINVAL, "problem " + std::to_string(i) + ": dt, dx (and alpha) must be finite, dx != 0");
  }
  auto* b = new (std::nothrow) swept_batch_s();
  if (!b) return bfail(SWEPT_ENOMEM, "host allocation failed");
  b->kind = kind;
  b->dtype = dtype;
  b->nprob = nprob;
  b->steps = steps;
  b->n.assign(n, n + nprob);
  b->dt.assign(dt, dt + nprob);
  b->dx.assign(dx, dx + nprob);
  b->alpha = kind == SWEPT_HEAT_FTCS ? std::vector<double>(alpha, alpha + nprob) : std::vector<double>((size_t)nprob, 0.0);
  b->offsets.resize((size_t)nprob);
  int64_t off = 0;
  for (int32_t i = 0; i < nprob; ++i) {
    b->offsets[(size_t)i] = off;
    off += n[i];
  }
  b->total_points = off;
  b->poison = swept::debug_poison_requested();
  // queue order: largest first (ties by input index)
  b->order.resize((size_t)nprob);
  std::iota(b->order.begin(), b->order.end(), 0);
  std::stable_sort(b->order.begin(), b->order.end(), [&](int32_t x, int32_t y) { return n[x] > n[y]; });

  hipError_t e = hipGetDevice(&b->device);
  if (e != hipSuccess) {
    delete b;
    return bhip(e, "hipGetDevice");
  }
  int rc = build_tiling(b, b->engine, points_per_lane(kind, b->engine));
  if (rc != SWEPT_OK) {
    batch_free(b);
    return rc;
  }
  e = hipMalloc(reinterpret_cast<void**>(&b->queue), sizeof(int));
  if (e != hipSuccess) {
    batch_free(b);
    return bfail(SWEPT_ENOMEM, std::string("hipMalloc(batch queue): ") + hipGetErrorString(e));
  }
  e = size_grid(b);
  if (e != hipSuccess) {
    batch_free(b);
    return bhip(e, "occupancy query");
  }
  *out = b;
  return SWEPT_OK;
}

int swept_batch_set_engine(swept_batch b, int engine) {
  if (!b) return bfail(SWEPT_EINVAL, "batch must not be NULL");
  if (engine == SWEPT_ENGINE_LDS) return bfail(SWEPT_EUNSUPPORTED, "the batched kernel has no LDS engine");
  if (engine != SWEPT_ENGINE_AUTO && engine != SWEPT_ENGINE_WAVE && engine != SWEPT_ENGINE_COMPACT &&
      engine != SWEPT_ENGINE_RESIDENT)
    return bfail(SWEPT_EINVAL, "unknown engine");
  if (engine == b->engine) return SWEPT_OK;
  if (engine == SWEPT_ENGINE_WAVE) {
    // the register engine's tile halves are whole lanes of 16 points
    for (int32_t i = 0; i < b->nprob; ++i)
      if (b->n[(size_t)i] % 16 != 0)
        return bfail(SWEPT_EUNSUPPORTED, "problem " + std::to_string(i) +
                                             ": the register engine needs n to be a multiple of 16");
  }
  int prev = -1;
  hipError_t e = hipGetDevice(&prev);
  if (e == hipSuccess && prev != b->device) e = hipSetDevice(b->device);
  if (e != hipSuccess) return bhip(e, "hipSetDevice");
  const int old_engine = b->engine;
  // the grids' split between the kernels and the tiling follow the engine;
  // the slots hold no state between runs
  int rc = build_tiling(b, engine, points_per_lane(b->kind, engine));
  if (rc == SWEPT_OK) {
    b->engine = engine;
    e = size_grid(b);
    if (e != hipSuccess) {
      b->engine = old_engine;
      rc = bhip(e, "occupancy query");
      (void)build_tiling(b, old_engine, points_per_lane(b->kind, old_engine));
    }
    drop_graph(b);
  }
  if (prev != b->device) (void)hipSetDevice(prev);
  return rc;
}

int swept_batch_run(swept_batch b, void* u, int use_graph, void* stream) {
  if (!b) return bfail(SWEPT_EINVAL, "batch must not be NULL");
  if (!u) return bfail(SWEPT_EINVAL, "u must not be NULL");
  if (b->steps == 0) return SWEPT_OK;
  int prev = -1;
  hipError_t e = hipGetDevice(&prev);
  if (e != hipSuccess) return bhip(e, "hipGetDevice");
  if (prev != b->device && (e = hipSetDevice(b->device)) != hipSuccess) return bhip(e, "hipSetDevice");
  hipStream_t st = static_cast<hipStream_t>(stream);
  int rc = SWEPT_OK;
  if (!use_graph) {
    e = enqueue_batch(b, u, st);
    if (e != hipSuccess) rc = bhip(e, "batch launch");
  } else {
    if (b->exec && b->graph_u != u) drop_graph(b);
    if (!b->exec) {
      if (!b->cap_stream) e = hipStreamCreate(&b->cap_stream);
      if (e == hipSuccess) e = hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal);
      if (e == hipSuccess) {
        hipError_t le = enqueue_batch(b, u, b->cap_stream);
        e = hipStreamEndCapture(b->cap_stream, &b->graph);
        if (le != hipSuccess) e = le;
      }
      if (e == hipSuccess) e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
      if (e != hipSuccess) {
        if (b->graph) (void)hipGraphDestroy(b->graph);
        b->graph = nullptr;
        b->exec = nullptr;
        rc = bhip(e, "batch graph capture");
      } else {
        b->graph_u = u;
      }
    }
    if (rc == SWEPT_OK) {
      e = hipGraphLaunch(b->exec, st);
      if (e != hipSuccess) rc = bhip(e, "hipGraphLaunch");
    }
  }
  if (rc == SWEPT_OK && (b->checks & SWEPT_CHECK_NONFINITE)) {
    int bad = 0;
    e = hipStreamSynchronize(st);
    if (e == hipSuccess) e = hipMemcpy(&bad, b->flag, sizeof(int), hipMemcpyDeviceToHost);
    if (e != hipSuccess)
      rc = bhip(e, "non-finite check");
    else if (bad)
      rc = bfail(SWEPT_ENONFINITE, "a grid holds a non-finite value after the run");
  }
  if (prev != b->device) (void)hipSetDevice(prev);
  return rc;
}

int swept_batch_set_checks(swept_batch b, int flags) {
  if (!b) return bfail(SWEPT_EINVAL, "batch must not be NULL");
  if (flags & ~SWEPT_CHECK_NONFINITE) return bfail(SWEPT_EINVAL, "unknown check flags");
  if (flags == b->checks) return SWEPT_OK;
  if ((flags & SWEPT_CHECK_NONFINITE) && !b->flag) {
    int prev = -1;
    hipError_t e = hipGetDevice(&prev);
    if (e == hipSuccess && prev != b->device) e = hipSetDevice(b->device);
    if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&b->flag), sizeof(int));
    if (prev >= 0 && prev != b->device) (void)hipSetDevice(prev);
    if (e != hipSuccess) {
      b->flag = nullptr;
      return bfail(SWEPT_ENOMEM, std::string("hipMalloc(check flag): ") + hipGetErrorString(e));
    }
  }
  b->checks = flags;
  drop_graph(b);  // the captured launches include (or not) the check
  return SWEPT_OK;
}

int swept_batch_info(swept_batch b, int64_t* total_points, int64_t* offsets, size_t* workspace_bytes, int* grid) {
  if (!b) return bfail(SWEPT_EINVAL, "batch must not be NULL");
  if (total_points) *total_points = b->total_points;
  if (offsets) std::copy(b->offsets.begin(), b->offsets.end(), offsets);
  if (workspace_bytes) *workspace_bytes = b->slots_bytes;
  if (grid) *grid = b->grid;
  return SWEPT_OK;
}

void swept_batch_destroy(swept_batch b) {
  if (!b) return;
  const int dev = b->device;
  int prev = -1;
  const bool ok = hipGetDevice(&prev) == hipSuccess;
  if (ok && prev != dev) (void)hipSetDevice(dev);
  batch_free(b);
  if (ok && prev >= 0 && prev != dev) (void)hipSetDevice(prev);
}

}  // extern "C"
