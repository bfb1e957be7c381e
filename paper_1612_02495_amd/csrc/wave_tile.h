// One swept phase of one tile held in the registers of one wave64: the
// device code shared by the single-grid wave engine (phase_wave.hip) and the
// batched persistent kernel (batch.hip).
//
// Layout.  Lane L owns the P contiguous tile points L*P .. L*P+P-1.  A tile is
// kL + kR lanes wide (kL, kR <= 32): w = (kL + kR) P points, its inner seam at
// a = kL P.  The V part fills the gap centred on the inner seam; the Lambda
// part climbs the triangle between the tile ends; the flat top of a
// trapezoid is split at the inner seam (Sec. 4.2, 4.3).  Lanes >= kL + kR,
// when there are any, carry don't-care values.
//
// Every tier is computed across the whole wave; the part of a tier the swept
// rule leaves unknown holds don't-care data that no valid point consumes.
// Neighbours across lanes come from DPP wave shifts.  The edge bands move s
// points per tier -- one lane every B = P/s tiers -- so the tier loop is
// unrolled in blocks of B tiers, inside which every band point has a
// compile-time register index and one of two block-uniform owner lanes:
// inserting (V) or collecting (Lambda) a band value is one v_cndmask per
// 32-bit word under a lane mask.
//
// Edge slots hold one side of a producer tile, position-major [p][tier & 1]
// (every point lies in the outermost 2s band of exactly two consecutive
// tiers; a trapezoid's flat top is the value at its top tier):
//   producer left side   x in [0, a + s)      -> p = x
//   producer right side  x in [a - s, w)      -> p = x - a + s
//   consumer left input  x in [-s, a)         -> p = x + s
//   consumer right input x in [a, w + s)      -> p = x - a
// Slots hold 64 P + 2 s values (kL, kR <= 32).
#pragma once

#include "internal.h"

namespace swept {
namespace wave {

constexpr int kDppWaveShr1 = 0x138;  // lane i <- lane i-1
constexpr int kDppWaveShl1 = 0x130;  // lane i <- lane i+1

// Cross-lane move where the lane without a source reads zero.
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

// Select by value (a conditional on two array elements would otherwise select
// between their addresses and keep the arrays out of registers).
template <typename T>
__device__ __forceinline__ T pick(bool c, T a, T b) {
  return c ? a : b;
}

// Lanes [lo, hi) of a wave64 as a 64-bit lane mask (bit i = lane i), clipped
// to the wave.  With compile-time bounds this folds to a constant.
__host__ __device__ constexpr uint64_t range_bits(int lo, int hi) {
  lo = lo < 0 ? 0 : lo;
  hi = hi > 64 ? 64 : hi;
  if (hi <= lo) return 0;
  const uint64_t below_hi = hi >= 64 ? ~0ull : ((1ull << hi) - 1);
  return below_hi & ~((1ull << lo) - 1);
}

// This lane's bit of a wave-uniform lane mask.  A constant mask becomes a
// scalar operand of the select itself: no per-lane compare is issued.
__device__ __forceinline__ bool lanes(uint64_t m) { return __builtin_amdgcn_inverse_ballot_w64(m); }

// Halo values of lane L's neighbours: lo[i] = point L*P - S + i, hi[i] =
// point L*P + P + i.  With TIPS, lane 0's lo and lane (kE-1)'s hi are the
// triangle tips beyond the tile ends.
template <typename T, int P, int S, bool TIPS>
__device__ __forceinline__ void halos(const T (&src)[P], const T (&tipL)[S], const T (&tipR)[S], bool first,
                                      bool last, T (&lo)[S], T (&hi)[S]) {
#pragma unroll
  for (int i = 0; i < S; ++i) {
    lo[i] = dpp_move0<kDppWaveShr1>(src[P - S + i]);
    hi[i] = dpp_move0<kDppWaveShl1>(src[i]);
    if constexpr (TIPS) {
      lo[i] = pick(first, tipL[i], lo[i]);
      hi[i] = pick(last, tipR[i], hi[i]);
    }
  }
}

// Value at lane-relative offset o in [-S, P + S) of a row with halos.
template <typename T, int P, int S>
__device__ __forceinline__ T at(const T (&row)[P], const T (&lo)[S], const T (&hi)[S], int o) {
  if (o < 0) return lo[o + S];
  if (o >= P) return hi[o - P];
  return row[o];
}

// Lanes holding an end of an insulated rod (heat only): `left` marks the
// lane whose first point is node 0, `right` the lane whose last point is node
// n-1.  Their missing neighbour is the mirror ghost about the end node.
struct Ends {
  bool left = false;
  bool right = false;
};

// Advance the tile from tier t to tier t+1.  Heat: one row A.  KS: A holds
// even tiers (finals), Q odd tiers (predictors).  INS (heat): the lanes of
// `e` take the mirror ghost at the rod's ends, u_{-1} = u_1, u_n = u_{n-2}.
template <int KIND, typename T, int P, bool TIPS, bool INS = false>
__device__ __forceinline__ void tier(T (&A)[P], T (&Q)[P], bool t1_odd, const T (&tipL)[Radius<KIND>::value],
                                     const T (&tipR)[Radius<KIND>::value], bool first, bool last,
                                     const Consts<T>& k, Ends e = Ends{}) {
  constexpr int S = Radius<KIND>::value;
  static_assert(!INS || (KIND == kHeat && P >= 2), "insulated ends: heat, two or more points per lane");
  T lo[S], hi[S];
  if constexpr (KIND == kHeat) {
    halos<T, P, S, TIPS>(A, tipL, tipR, first, last, lo, hi);
    T prev = lo[0];
    if constexpr (INS) prev = pick(e.left, A[1], prev);
#pragma unroll
    for (int r = 0; r < P; ++r) {
      T right = r == P - 1 ? hi[0] : A[r + 1];
      if constexpr (INS) {
        if (r == P - 1) right = pick(e.right, prev, right);
      }
      const T nv = heat_update(prev, A[r], right, k);
      prev = A[r];
      A[r] = nv;
    }
  } else if (t1_odd) {
    halos<T, P, S, TIPS>(A, tipL, tipR, first, last, lo, hi);
#pragma unroll
    for (int r = 0; r < P; ++r)
      Q[r] = ks_predictor(at<T, P, S>(A, lo, hi, r - 2), at<T, P, S>(A, lo, hi, r - 1), A[r],
                          at<T, P, S>(A, lo, hi, r + 1), at<T, P, S>(A, lo, hi, r + 2), k);
  } else {
    halos<T, P, S, TIPS>(Q, tipL, tipR, first, last, lo, hi);
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
// then compute tier t+1.  Left band of tier t: [a - S(t+2), a - S t), owned
// by lanes kL-1-b and kL-2-b; right band [a + S t, a + S(t+2)), lanes kL+b
// and kL+1+b.
template <int KIND, typename T, int P, bool FULL, bool TIPS>
__device__ __forceinline__ void v_block(T (&A)[P], T (&Q)[P], const T (&buf)[P][2], int b, int hv, int lane,
                                        int kL, bool first, bool last, const T (&tipL)[Radius<KIND>::value],
                                        const T (&tipR)[Radius<KIND>::value], const Consts<T>& k) {
  constexpr int S = Radius<KIND>::value;
  constexpr int B = P / S;
  const bool mL0 = lane == kL - 1 - b, mL1 = lane == kL - 2 - b;
  const bool mR0 = lane == kL + b, mR1 = lane == kL + 1 + b;
#pragma unroll
  for (int j = 0; j < B; ++j) {
    const int t = b * B + j;
    if (FULL || t < hv) {
      T(&row)[P] = KIND == kHeat ? A : row_of<T, P>(A, Q, j & 1);
#pragma unroll
      for (int i = 0; i < 2 * S; ++i) {
        const int ol = P - S * (j + 2) + i;  // offset from lane kL-1-b
        const int rl = (ol + P) % P;
        row[rl] = pick(ol < 0 ? mL1 : mL0, buf[rl][j & 1], row[rl]);
        const int orr = S * j + i;  // offset from lane kL+b
        const int rr = orr % P;
        row[rr] = pick(orr >= P ? mR1 : mR0, buf[rr][j & 1], row[rr]);
      }
      tier<KIND, T, P, TIPS>(A, Q, ((j + 1) & 1) != 0, tipL, tipR, first, last, k);
    }
  }
}

// Lambda part, tiers b*B .. b*B+B-1: collect the band values of tier t, then
// compute tier t+1 (skipped when it would be the empty top of a full
// triangle).  Left band of tier t: [S t, S t + 2S), lanes b and b+1; right
// band [w - S(t+2), w - S t), lanes kE-1-b and kE-2-b.
template <int KIND, typename T, int P, bool FULL>
__device__ __forceinline__ void l_block(T (&A)[P], T (&Q)[P], T (&buf)[P][2], int b, int hl, bool empty_top,
                                        int lane, int kE, const Consts<T>& k) {
  constexpr int S = Radius<KIND>::value;
  constexpr int B = P / S;
  const bool mL0 = lane == b, mL1 = lane == b + 1;
  const bool mR0 = lane == kE - 1 - b, mR1 = lane == kE - 2 - b;
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
        const int orr = P - S * (j + 2) + i;  // offset from lane kE-1-b
        const int rr = (orr + P) % P;
        buf[rr][j & 1] = pick(orr < 0 ? mR1 : mR0, row[rr], buf[rr][j & 1]);
      }
      if (FULL || t + 1 < hl || !empty_top)
        tier<KIND, T, P, false>(A, Q, ((j + 1) & 1) != 0, tip0, tip0, false, false, k);
    }
  }
}

// Tile geometry of one phase.
template <typename T>
struct Tile {
  int64_t origin;  // ring index of tile point 0
  T* sL;           // left edge slot (consumer left input / producer left side)
  T* sR;           // right edge slot
  int kL, kR;      // lanes left and right of the inner seam (1..32 each)
};

// MODE: 0 up-triangle (hv == 0), 1 diamond, 2 down-triangle (hl == 0),
// 3 any (decided at run time from hv and hl).
template <int KIND, typename T, int P, int MODE>
__device__ __forceinline__ void tile_phase(T* u, int64_t n, const Tile<T>& g, int hv, int hl, const Consts<T>& k,
                                           int lane) {
  constexpr int S = Radius<KIND>::value;
  constexpr int B = P / S;
  const int kL = g.kL;
  const int kE = g.kL + g.kR;
  const int w = kE * P;
  const int a = kL * P;
  const bool active = lane < kE;
  const bool has_v = MODE == 1 || MODE == 2 || (MODE == 3 && hv > 0);
  const bool has_l = MODE == 0 || MODE == 1 || (MODE == 3 && hl > 0);

  T A[P];
  T Q[P];
  T buf[P][2];
#pragma unroll
  for (int r = 0; r < P; ++r) {
    A[r] = T(0);
    Q[r] = T(0);
    buf[r][0] = T(0);
    buf[r][1] = T(0);
  }

  if (!has_v) {
    if (active) {
#pragma unroll
      for (int r = 0; r < P; ++r) {
        int64_t g2 = g.origin + lane * P + r;
        if (g2 >= n) g2 -= n;
        A[r] = u[g2];
      }
    }
  } else {
    // Incoming band values of this lane's points: left of the seam from the
    // left slot (p = x + S), right of it from the right slot (p = x - a).
    if (active) {
      const T* src = lane < kL ? g.sL + 2 * (lane * P + S) : g.sR + 2 * ((lane - kL) * P);
#pragma unroll
      for (int r = 0; r < P; ++r) {
        buf[r][0] = src[2 * r];
        buf[r][1] = src[2 * r + 1];
      }
    }
    // Triangle tips beyond the tile ends, used by the last V tier when the
    // gap reaches an end: points -S..-1 (left slot p < S) and w..w+S-1
    // (right slot p = kR P ..).
    T tipL[S], tipR[S];
    const int tp = (hv - 1) & 1;
#pragma unroll
    for (int i = 0; i < S; ++i) {
      tipL[i] = g.sL[2 * i + tp];
      tipR[i] = g.sR[2 * (g.kR * P + i) + tp];
    }
    const bool first = lane == 0;
    const bool last = lane == kE - 1;
    const int nb = (hv + B - 1) / B;
    for (int b = 0; b < nb - 1; ++b)
      v_block<KIND, T, P, true, false>(A, Q, buf, b, hv, lane, kL, first, last, tipL, tipR, k);
    v_block<KIND, T, P, false, true>(A, Q, buf, nb - 1, hv, lane, kL, first, last, tipL, tipR, k);
    // flat tops of the producer trapezoids: tile points outside the gap
    if (S * hv < a || S * hv < w - a) {
#pragma unroll
      for (int r = 0; r < P; ++r) {
        const int x = lane * P + r;
        if (x < a - S * hv || x >= a + S * hv) A[r] = pick((hv & 1) != 0, buf[r][1], buf[r][0]);
      }
    }
  }

  if (!has_l) {
    if (active) {
#pragma unroll
      for (int r = 0; r < P; ++r) {
        int64_t g2 = g.origin + lane * P + r;
        if (g2 >= n) g2 -= n;
        u[g2] = A[r];
      }
    }
    return;
  }
#pragma unroll
  for (int r = 0; r < P; ++r) {
    buf[r][0] = T(0);
    buf[r][1] = T(0);
  }
  const bool empty_top = 2 * S * hl >= w;
  const int nb = (hl + B - 1) / B;
  for (int b = 0; b < nb - 1; ++b) l_block<KIND, T, P, true>(A, Q, buf, b, hl, empty_top, lane, kE, k);
  l_block<KIND, T, P, false>(A, Q, buf, nb - 1, hl, empty_top, lane, kE, k);
  if (!empty_top) {
#pragma unroll
    for (int r = 0; r < P; ++r) {
      const int x = lane * P + r;
      if (x >= S * hl && x < w - S * hl) {
        // register indices stay compile-time: select on the parity instead
        if (hl & 1)
          buf[r][1] = A[r];
        else
          buf[r][0] = A[r];
      }
    }
  }
  // Outgoing slots: left side p = x for x < a + S, right side p = x - a + S
  // for x >= a - S (the tip points go to both).
  if (active) {
    T* dst = lane < kL ? g.sL + 2 * (lane * P) : g.sR + 2 * ((lane - kL) * P + S);
#pragma unroll
    for (int r = 0; r < P; ++r) {
      dst[2 * r] = buf[r][0];
      dst[2 * r + 1] = buf[r][1];
    }
  }
  if (lane == kL - 1) {
#pragma unroll
    for (int r = P - S; r < P; ++r) {
      g.sR[2 * (r - P + S)] = buf[r][0];
      g.sR[2 * (r - P + S) + 1] = buf[r][1];
    }
  } else if (lane == kL) {
#pragma unroll
    for (int r = 0; r < S; ++r) {
      g.sL[2 * (a + r)] = buf[r][0];
      g.sL[2 * (a + r) + 1] = buf[r][1];
    }
  }
}

}  // namespace wave
}  // namespace swept
