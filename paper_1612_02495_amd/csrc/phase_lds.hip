// LDS engine: one thread block per tile ("node", Sec. 4.2), the tile kept in
// two LDS rows that alternate between even and odd tiers (the two-row matrix
// of Sec. 4.2; for KS the odd row holds predictors and the even row finals,
// Sec. 4.3).  Rows carry s extra cells on each side for the triangle tips.
//
// Phase = V (hv tiers) then Lambda (hl tiers), see PhaseArgs.
//
// Edge-slot layout (shared with the wave engine).  A slot holds one side of a
// producer tile: position-major entries [p][t], t = tier & 1, because every
// position appears in the outermost 2s band of exactly two consecutive tiers
// (and the flat top of a trapezoid is the value at tier hl).
//   producer left side:   tile position x in [0, w/2 + s)   -> p = x
//   producer right side:  tile position x in [w/2 - s, w)   -> p = x - w/2 + s
//   consumer left input:  tile position x in [-s, w/2)      -> p = x + s
//   consumer right input: tile position x in [w/2, w + s)   -> p = x - w/2
// Parity-0 tile j owns slots A[j] (left) and B[j] (right); parity-1 tile j
// owns B[j] (left) and A[(j+1) mod nt] (right).  A tile reads both of its
// slots completely before it writes them, and no other tile touches them
// during the phase, so the strips are updated in place.
#include "internal.h"
#include "poison.h"

namespace swept {
namespace {

constexpr int kLdsThreads = 256;

template <int KIND, typename T>
__device__ __forceinline__ void tier_update(T* __restrict__ dst, const T* __restrict__ src, int x, int tier,
                                            const Consts<T>& k) {
  if constexpr (KIND == kHeat) {
    dst[x] = heat_update(src[x - 1], src[x], src[x + 1], k);
  } else {
    if (tier & 1)
      dst[x] = ks_predictor(src[x - 2], src[x - 1], src[x], src[x + 1], src[x + 2], k);
    else
      dst[x] = ks_final(dst[x], src[x - 2], src[x - 1], src[x], src[x + 1], src[x + 2], k);
  }
}

// ROLE only names the launch for profilers (0 up-triangle, 1 diamond,
// 2 down-triangle); the phase shape comes from hv and hl.
template <int KIND, typename T, int ROLE>
__global__ void __launch_bounds__(kLdsThreads)
phase_lds_kernel(T* __restrict__ u, T* __restrict__ slots, int64_t n, int w, int64_t nt, int parity,
                 int hv, int hl, Consts<T> k, int poison) {
  constexpr int S = Radius<KIND>::value;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* smem = reinterpret_cast<T*>(smem_raw);
  const int rowlen = w + 2 * S;
  const int slen = slot_values(w, S);
  if (poison) {
    poison_lds(smem, 2 * rowlen + 2 * slen, (int)threadIdx.x, (int)blockDim.x);
    __syncthreads();
  }
  T* row[2] = {smem + S, smem + rowlen + S};  // index x in [-S, w + S)
  T* inL = smem + 2 * rowlen;
  T* inR = inL + slen;

  const int tid = threadIdx.x;
  const int nthr = blockDim.x;
  const int64_t j = blockIdx.x;
  const int half = w >> 1;
  const int64_t origin = j * (int64_t)w + (parity ? half : 0);
  T* slotA = slots;
  T* slotB = slots + nt * (int64_t)slen;
  T* sL = parity ? slotB + j * slen : slotA + j * slen;
  T* sR = parity ? slotA + ((j + 1) % nt) * slen : slotB + j * slen;

  // ------------------------------------------------------------ V part --
  if (hv == 0) {
    for (int x = tid; x < w; x += nthr) {
      int64_t g = origin + x;
      if (g >= n) g -= n;
      row[0][x] = u[g];
    }
  } else {
    for (int i = tid; i < slen; i += nthr) {
      inL[i] = sL[i];
      inR[i] = sR[i];
    }
    __syncthreads();
    // tier-0 edge bands: left [w/2 - 2S, w/2), right [w/2, w/2 + 2S)
    if (tid < 2 * S) {
      const int x = half - 2 * S + tid;
      row[0][x] = inL[2 * (x + S)];
    } else if (tid < 4 * S) {
      const int x = half + (tid - 2 * S);
      row[0][x] = inR[2 * (x - half)];
    }
  }
  __syncthreads();

  for (int kk = 0; kk < hv; ++kk) {
    const int t1 = kk + 1;
    const T* src = row[kk & 1];
    T* dst = row[t1 & 1];
    // fill the gap of tier t1: [w/2 - S t1, w/2 + S t1)
    const int lo = half - S * t1;
    const int hi = half + S * t1;
    for (int x = lo + tid; x < hi; x += nthr) tier_update<KIND>(dst, src, x, t1, k);
    if (t1 < hv) {
      // edge bands of tier t1 from the incoming slots
      if (tid < 2 * S) {
        const int x = lo - 2 * S + tid;
        dst[x] = inL[2 * (x + S) + (t1 & 1)];
      } else if (tid < 4 * S) {
        const int x = hi + (tid - 2 * S);
        dst[x] = inR[2 * (x - half) + (t1 & 1)];
      }
    } else {
      // flat tops of the two producer trapezoids (empty for full triangles)
      for (int x = tid; x < lo; x += nthr) dst[x] = inL[2 * (x + S) + (t1 & 1)];
      for (int x = hi + tid; x < w; x += nthr) dst[x] = inR[2 * (x - half) + (t1 & 1)];
    }
    __syncthreads();
  }

  // ------------------------------------------------------- Lambda part --
  const int base = hv & 1;  // row holding tier hv (the full row)
  if (hl == 0) {
    const T* full = row[base];
    for (int x = tid; x < w; x += nthr) {
      int64_t g = origin + x;
      if (g >= n) g -= n;
      u[g] = full[x];
    }
    return;
  }
  for (int kk = 0; kk < hl; ++kk) {
    const T* src = row[(base + kk) & 1];
    T* dst = row[(base + kk + 1) & 1];
    // edge bands of tier kk: left [S kk, S kk + 2S), right [w - S kk - 2S, w - S kk)
    if (tid < 2 * S) {
      const int x = S * kk + tid;
      sL[2 * x + (kk & 1)] = src[x];
    } else if (tid < 4 * S) {
      const int x = w - S * kk - 2 * S + (tid - 2 * S);
      sR[2 * (x - half + S) + (kk & 1)] = src[x];
    }
    const int t1 = kk + 1;
    for (int x = S * t1 + tid; x < w - S * t1; x += nthr) tier_update<KIND>(dst, src, x, hv + t1, k);
    __syncthreads();
  }
  // flat top of tier hl (empty when hl = w/(2S))
  const T* top = row[(base + hl) & 1];
  for (int x = S * hl + tid; x < w - S * hl; x += nthr) {
    if (x < half)
      sL[2 * x + (hl & 1)] = top[x];
    else
      sR[2 * (x - half + S) + (hl & 1)] = top[x];
  }
}

}  // namespace

template <int KIND, typename T>
size_t phase_lds_bytes(int w) {
  constexpr int S = Radius<KIND>::value;
  return (size_t)(2 * (w + 2 * S) + 2 * slot_values(w, S)) * sizeof(T);
}

int phase_lds_threads(int w) { return w >= kLdsThreads ? kLdsThreads : ((w + 63) / 64) * 64; }

template <int KIND, typename T>
hipError_t launch_phase_lds(const PhaseArgs& a, const Consts<T>& k, hipStream_t st) {
  const int threads = phase_lds_threads(a.w);
  const size_t lds = phase_lds_bytes<KIND, T>(a.w);
  auto kern = a.hv == 0 ? phase_lds_kernel<KIND, T, 0>
              : (a.hl == 0 ? phase_lds_kernel<KIND, T, 2> : phase_lds_kernel<KIND, T, 1>);
  hipLaunchKernelGGL(kern, dim3((unsigned)a.nt), dim3(threads), lds, st, static_cast<T*>(a.u),
                     static_cast<T*>(a.slots), a.n, a.w, a.nt, a.parity, a.hv, a.hl, k, a.poison);
  return hipGetLastError();
}

#define SWEPT_INST_LDS(KIND, T)                                                                  \
  template size_t phase_lds_bytes<KIND, T>(int);                                                 \
  template hipError_t launch_phase_lds<KIND, T>(const PhaseArgs&, const Consts<T>&, hipStream_t);
SWEPT_INST_LDS(kHeat, float)
SWEPT_INST_LDS(kHeat, double)
SWEPT_INST_LDS(kKS, float)
SWEPT_INST_LDS(kKS, double)
#undef SWEPT_INST_LDS

}  // namespace swept
