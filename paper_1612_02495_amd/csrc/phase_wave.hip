// Wave-resident engine: one wave64 per tile ("node", Sec. 4.2), the tile held
// in registers -- lane L owns the P contiguous points L*P .. L*P+P-1, so a
// tile is w = 64*P points -- and no LDS or barrier in the tier loop.
//
// Every tier is computed across the whole tile; the two lanes' worth of
// values the swept rule leaves unknown at a tier simply hold don't-care data
// that is never consumed by a valid point.  Neighbour values across lanes come
// from DPP wave shifts (wave_shr:1 / wave_shl:1), the wave64 analogue of the
// warp shuffles of the register-only variant (Sec. 4.5).
//
// The edge bands (Sec. 4.2) move s points per tier, i.e. exactly one lane's
// worth of points every B = P/s tiers.  The tier loop is therefore unrolled in
// blocks of B tiers: inside a block every band point has a compile-time
// register index and one of two block-uniform owner lanes, so inserting
// (V part) or collecting (Lambda part) a band value is one v_cndmask per
// 32-bit word under a lane mask.  Each lane preloads, with coalesced vector
// loads, the two band values of each of its own points (every point lies in
// the band of exactly two consecutive tiers), and collects its outgoing band
// values in the same registers before one coalesced store.
//
// Edge-slot layout and tile/slot ownership are those of the LDS engine
// (phase_lds.hip), so the two engines can run alternate phases of one run.
#include "internal.h"

namespace swept {
namespace {

constexpr int kDppWaveShr1 = 0x138;  // lane i <- lane i-1
constexpr int kDppWaveShl1 = 0x130;  // lane i <- lane i+1

// Cross-lane move; lanes without a source lane (lane 0 for shr, lane 63 for
// shl) receive `edge`.
template <int CTRL>
__device__ __forceinline__ double dpp_move(double v, double edge) {
  const long long x = __double_as_longlong(v);
  const long long e = __double_as_longlong(edge);
  const int lo = __builtin_amdgcn_update_dpp((int)e, (int)x, CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp((int)(e >> 32), (int)(x >> 32), CTRL, 0xf, 0xf, false);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}
template <int CTRL>
__device__ __forceinline__ float dpp_move(float v, float edge) {
  return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(edge), __float_as_int(v), CTRL, 0xf, 0xf, false));
}
// Same move where the edge lane does not matter (it reads zero).
template <int CTRL>
__device__ __forceinline__ double dpp_move0(double v) {
  const long long x = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_mov_dpp((int)x, CTRL, 0xf, 0xf, true);
  const int hi = __builtin_amdgcn_mov_dpp((int)(x >> 32), CTRL, 0xf, 0xf, true);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}
template <int CTRL>
__device__ __forceinline__ float dpp_move0(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xf, 0xf, true));
}

// Halo values of lane L's neighbours: lo[i] = point L*P - S + i, hi[i] = point L*P + P + i.
template <typename T, int P, int S, bool TIPS>
__device__ __forceinline__ void halos(const T (&src)[P], const T (&tipL)[S], const T (&tipR)[S], T (&lo)[S],
                                      T (&hi)[S]) {
#pragma unroll
  for (int i = 0; i < S; ++i) {
    if constexpr (TIPS) {
      lo[i] = dpp_move<kDppWaveShr1>(src[P - S + i], tipL[i]);
      hi[i] = dpp_move<kDppWaveShl1>(src[i], tipR[i]);
    } else {
      lo[i] = dpp_move0<kDppWaveShr1>(src[P - S + i]);
      hi[i] = dpp_move0<kDppWaveShl1>(src[i]);
    }
  }
}

// Select by value (a conditional on two array elements would otherwise select
// between their addresses and keep the arrays out of registers).
template <typename T>
__device__ __forceinline__ T pick(bool c, T a, T b) {
  return c ? a : b;
}

// Value at lane-relative offset o in [-S, P + S) of a row with halos.
template <typename T, int P, int S>
__device__ __forceinline__ T at(const T (&row)[P], const T (&lo)[S], const T (&hi)[S], int o) {
  if (o < 0) return lo[o + S];
  if (o >= P) return hi[o - P];
  return row[o];
}

// Advance the tile from tier t to tier t+1 (t1 = t+1).  Heat: one row A.
// KS: A holds even tiers (finals), Q odd tiers (predictors).
template <int KIND, typename T, int P, bool TIPS>
__device__ __forceinline__ void tier(T (&A)[P], T (&Q)[P], bool t1_odd, const T (&tipL)[Radius<KIND>::value],
                                     const T (&tipR)[Radius<KIND>::value], const Consts<T>& k) {
  constexpr int S = Radius<KIND>::value;
  T lo[S], hi[S];
  if constexpr (KIND == kHeat) {
    halos<T, P, S, TIPS>(A, tipL, tipR, lo, hi);
    T prev = lo[0];
#pragma unroll
    for (int r = 0; r < P; ++r) {
      const T right = r == P - 1 ? hi[0] : A[r + 1];
      const T nv = heat_update(prev, A[r], right, k);
      prev = A[r];
      A[r] = nv;
    }
  } else if (t1_odd) {
    halos<T, P, S, TIPS>(A, tipL, tipR, lo, hi);
#pragma unroll
    for (int r = 0; r < P; ++r)
      Q[r] = ks_predictor(at<T, P, S>(A, lo, hi, r - 2), at<T, P, S>(A, lo, hi, r - 1), A[r],
                          at<T, P, S>(A, lo, hi, r + 1), at<T, P, S>(A, lo, hi, r + 2), k);
  } else {
    halos<T, P, S, TIPS>(Q, tipL, tipR, lo, hi);
#pragma unroll
    for (int r = 0; r < P; ++r)
      A[r] = ks_final(A[r], at<T, P, S>(Q, lo, hi, r - 2), at<T, P, S>(Q, lo, hi, r - 1), Q[r],
                      at<T, P, S>(Q, lo, hi, r + 1), at<T, P, S>(Q, lo, hi, r + 2), k);
  }
}

template <typename T, int P>
__device__ __forceinline__ T (&row_of(T (&A)[P], T (&Q)[P], bool odd))[P] {
  return odd ? Q : A;
}

// V part, tiers b*B .. b*B+B-1: insert the incoming band values of tier t,
// then compute tier t+1.  Left band of tier t occupies tile points
// [w/2 - S(t+2), w/2 - S t), right band [w/2 + S t, w/2 + S(t+2)).
template <int KIND, typename T, int P, bool FULL, bool TIPS>
__device__ __forceinline__ void v_block(T (&A)[P], T (&Q)[P], const T (&buf)[P][2], int b, int hv, int lane,
                                        const T (&tipL)[Radius<KIND>::value],
                                        const T (&tipR)[Radius<KIND>::value], const Consts<T>& k) {
  constexpr int S = Radius<KIND>::value;
  constexpr int B = P / S;
  const bool mL0 = lane == 31 - b, mL1 = lane == 30 - b;
  const bool mR0 = lane == 32 + b, mR1 = lane == 33 + b;
#pragma unroll
  for (int j = 0; j < B; ++j) {
    const int t = b * B + j;
    if (FULL || t < hv) {
      T(&row)[P] = KIND == kHeat ? A : row_of<T, P>(A, Q, j & 1);
#pragma unroll
      for (int i = 0; i < 2 * S; ++i) {
        const int ol = P - S * (j + 2) + i;  // offset from lane (31-b)
        const int rl = (ol + P) % P;
        row[rl] = pick(ol < 0 ? mL1 : mL0, buf[rl][j & 1], row[rl]);
        const int orr = S * j + i;  // offset from lane (32+b)
        const int rr = orr % P;
        row[rr] = pick(orr >= P ? mR1 : mR0, buf[rr][j & 1], row[rr]);
      }
      tier<KIND, T, P, TIPS>(A, Q, ((j + 1) & 1) != 0, tipL, tipR, k);
    }
  }
}

// Lambda part, tiers b*B .. b*B+B-1: collect the band values of tier t, then
// compute tier t+1 (skipped when it is the empty top of a full triangle).
// Left band of tier t: [S t, S t + 2S); right band: [w - S t - 2S, w - S t).
template <int KIND, typename T, int P, bool FULL>
__device__ __forceinline__ void l_block(T (&A)[P], T (&Q)[P], T (&buf)[P][2], int b, int hl, bool pure, int lane,
                                        const Consts<T>& k) {
  constexpr int S = Radius<KIND>::value;
  constexpr int B = P / S;
  const bool mL0 = lane == b, mL1 = lane == b + 1;
  const bool mR0 = lane == 63 - b, mR1 = lane == 62 - b;
  const T tip0[S] = {};
#pragma unroll
  for (int j = 0; j < B; ++j) {
    const int t = b * B + j;
    if (FULL || t < hl) {
      T(&row)[P] = KIND == kHeat ? A : row_of<T, P>(A, Q, j & 1);
#pragma unroll
      for (int i = 0; i < 2 * S; ++i) {
        const int ol = S * j + i;  // offset from lane b
        const int rl = ol % P;
        buf[rl][j & 1] = pick(ol >= P ? mL1 : mL0, row[rl], buf[rl][j & 1]);
        const int orr = P - S * (j + 2) + i;  // offset from lane (63-b)
        const int rr = (orr + P) % P;
        buf[rr][j & 1] = pick(orr < 0 ? mR1 : mR0, row[rr], buf[rr][j & 1]);
      }
      if (FULL || t + 1 < hl || !pure) tier<KIND, T, P, false>(A, Q, ((j + 1) & 1) != 0, tip0, tip0, k);
    }
  }
}

// ROLE: 0 up-triangle (hv == 0), 1 diamond, 2 down-triangle (hl == 0).
template <int KIND, typename T, int P, int ROLE>
__global__ void __launch_bounds__(64)
phase_wave_kernel(T* u, T* slots, int64_t n, int64_t nt, int parity, int hv, int hl, Consts<T> k) {
  constexpr int S = Radius<KIND>::value;
  constexpr int W = 64 * P;
  constexpr int HALF = 32 * P;
  constexpr int B = P / S;
  constexpr int SLEN = W + 2 * S;
  constexpr int HP = KIND == kHeat ? W / 2 : W / 4;  // tiers of a full triangle
  const int lane = threadIdx.x;
  const int64_t j = blockIdx.x;
  const int64_t origin = j * (int64_t)W + (parity ? HALF : 0);
  T* sL = parity ? slots + (nt + j) * SLEN : slots + j * SLEN;
  T* sR = parity ? slots + ((j + 1) % nt) * SLEN : slots + (nt + j) * SLEN;

  T A[P];
  T Q[P];
  T buf[P][2];
#pragma unroll
  for (int r = 0; r < P; ++r) {
    A[r] = T(0);
    Q[r] = T(0);
  }

  if constexpr (ROLE == 0) {
#pragma unroll
    for (int r = 0; r < P; ++r) {
      int64_t g = origin + lane * P + r;
      if (g >= n) g -= n;
      A[r] = u[g];
    }
  } else {
    // Incoming band values of this lane's points: left half from the left
    // slot (p = x + S), right half from the right slot (p = x - w/2).
    const T* src = lane < 32 ? sL + 2 * (lane * P + S) : sR + 2 * (lane * P - HALF);
#pragma unroll
    for (int r = 0; r < P; ++r) {
      buf[r][0] = src[2 * r];
      buf[r][1] = src[2 * r + 1];
    }
    // Triangle tips beyond the tile ends, needed by the last V tier of a
    // full diamond: points -S..-1 (left slot p < S) and w..w+S-1.
    T tipL[S], tipR[S];
    const int tp = (hv - 1) & 1;
#pragma unroll
    for (int i = 0; i < S; ++i) {
      tipL[i] = sL[2 * i + tp];
      tipR[i] = sR[2 * (HALF + i) + tp];
    }
    const int nb = (hv + B - 1) / B;
    for (int b = 0; b < nb - 1; ++b) v_block<KIND, T, P, true, false>(A, Q, buf, b, hv, lane, tipL, tipR, k);
    v_block<KIND, T, P, false, true>(A, Q, buf, nb - 1, hv, lane, tipL, tipR, k);
    if (hv < HP) {
      // flat tops of the producer trapezoids: tile points outside the gap
#pragma unroll
      for (int r = 0; r < P; ++r) {
        const int x = lane * P + r;
        if (x < HALF - S * hv || x >= HALF + S * hv) A[r] = pick((hv & 1) != 0, buf[r][1], buf[r][0]);
      }
    }
  }

  if constexpr (ROLE == 2) {
#pragma unroll
    for (int r = 0; r < P; ++r) {
      int64_t g = origin + lane * P + r;
      if (g >= n) g -= n;
      u[g] = A[r];
    }
  } else {
#pragma unroll
    for (int r = 0; r < P; ++r) {
      buf[r][0] = T(0);
      buf[r][1] = T(0);
    }
    const bool pure = hl == HP;
    const int nb = (hl + B - 1) / B;
    for (int b = 0; b < nb - 1; ++b) l_block<KIND, T, P, true>(A, Q, buf, b, hl, pure, lane, k);
    l_block<KIND, T, P, false>(A, Q, buf, nb - 1, hl, pure, lane, k);
    if (!pure) {
#pragma unroll
      for (int r = 0; r < P; ++r) {
        const int x = lane * P + r;
        if (x >= S * hl && x < W - S * hl) {
          // register indices stay compile-time: select on the parity instead
          if (hl & 1)
            buf[r][1] = A[r];
          else
            buf[r][0] = A[r];
        }
      }
    }
    // Outgoing slots: left side p = x for x < w/2 + S, right side
    // p = x - w/2 + S for x >= w/2 - S (the tip points go to both).
    T* dst = lane < 32 ? sL + 2 * (lane * P) : sR + 2 * (lane * P - HALF + S);
#pragma unroll
    for (int r = 0; r < P; ++r) {
      dst[2 * r] = buf[r][0];
      dst[2 * r + 1] = buf[r][1];
    }
    if (lane == 31) {
#pragma unroll
      for (int r = P - S; r < P; ++r) {
        sR[2 * (r - P + S)] = buf[r][0];
        sR[2 * (r - P + S) + 1] = buf[r][1];
      }
    } else if (lane == 32) {
#pragma unroll
      for (int r = 0; r < S; ++r) {
        sL[2 * (HALF + r)] = buf[r][0];
        sL[2 * (HALF + r) + 1] = buf[r][1];
      }
    }
  }
}

template <int KIND, typename T, int P>
hipError_t launch_p(const PhaseArgs& a, const Consts<T>& k, hipStream_t st) {
  auto kern = a.hv == 0 ? phase_wave_kernel<KIND, T, P, 0>
              : (a.hl == 0 ? phase_wave_kernel<KIND, T, P, 2> : phase_wave_kernel<KIND, T, P, 1>);
  hipLaunchKernelGGL(kern, dim3((unsigned)a.nt), dim3(64), 0, st, static_cast<T*>(a.u), static_cast<T*>(a.slots),
                     a.n, a.nt, a.parity, a.hv, a.hl, k);
  return hipGetLastError();
}

}  // namespace

bool wave_engine_supports(int kind, int w) {
  if (w % 64 != 0) return false;
  const int p = w / 64;
  if (kind == kHeat) return p == 2 || p == 4 || p == 8 || p == 16;
  return p == 4 || p == 8 || p == 16;
}

template <int KIND, typename T>
hipError_t launch_phase_wave(const PhaseArgs& a, const Consts<T>& k, hipStream_t st) {
  if (!wave_engine_supports(KIND, a.w)) return hipErrorInvalidValue;
  switch (a.w / 64) {
    case 2:
      if constexpr (KIND == kHeat) return launch_p<KIND, T, 2>(a, k, st);
      break;
    case 4:
      return launch_p<KIND, T, 4>(a, k, st);
    case 8:
      return launch_p<KIND, T, 8>(a, k, st);
    case 16:
      return launch_p<KIND, T, 16>(a, k, st);
    default:
      break;
  }
  return hipErrorInvalidValue;
}

template hipError_t launch_phase_wave<kHeat, float>(const PhaseArgs&, const Consts<float>&, hipStream_t);
template hipError_t launch_phase_wave<kHeat, double>(const PhaseArgs&, const Consts<double>&, hipStream_t);
template hipError_t launch_phase_wave<kKS, float>(const PhaseArgs&, const Consts<float>&, hipStream_t);
template hipError_t launch_phase_wave<kKS, double>(const PhaseArgs&, const Consts<double>&, hipStream_t);

}  // namespace swept
