// Swept adjoint of the periodic Kuramoto-Sivashinsky RK2 scheme: dJ/du_0
// for J a functional of u_T, for every grid of a batch, by a reverse swept
// sweep that recomputes each swept cycle from its checkpointed edge states.
//
// Scheme (Eq. KSDisc with the RK2 midpoint of Sec. 4.1 and the Appendix):
// q = u + (dt/2) f(u), u' = u + dt f(q), f the 5-point right-hand side.
// Reverse mode, from lambda' = dJ/du':
//   mu     = dt Jf(q)^T lambda'                  (dJ/dq)
//   lambda = (lambda' + mu) + (dt/2) Jf(u)^T mu   (dJ/du)
// Jf(v)^T w at point i only needs v_i and w at i-2 .. i+2:
//   (2 v_i / (4 dx)) (w_{i-1} - w_{i+1}) + (w_{i-1} + w_{i+1} - 2 w_i)/dx^2
//   + (w_{i-2} - 4 w_{i-1} + 6 w_i - 4 w_{i+1} + w_{i+2})/dx^4, negated,
// evaluated with per-neighbour coefficients in the fixed order w_{i-1},
// w_{i+1}, w_i, w_{i-2}, w_{i+2}: the first product rounded, each later one
// fused into the running sum.  The even-tier combination
// (lambda' + mu) + (dt/2) g is one fused multiply-add on the rounded sum.
//
// In tier terms (tier 2m = u after m steps, tier 2m+1 = predictor) the
// adjoint at tier d needs the adjoint at tier d+1 within two points and, for
// even d, its own point at tier d+2: the transpose of the forward tier rule
// (Sec. 4.3), with time reversed.  So the reverse sweep walks each swept
// region top-down over the same tiles, with the same edge bands moving the
// other way.
//
// Tiling.  Tiles of w = 64 points, one point per lane of one wave64, full
// (pure) phases of h = w/4 = 16 tiers (8 steps); the T mod 8 leading steps
// run with the classic scheme and keep their states.  Forward: phase p
// writes its edge bands (the 4 outermost points per side and tier) into
// checkpoint p.  Reverse, for p = K .. 0, one launch per phase: every tile
//   1. recomputes its region (V then Lambda) from checkpoint p-1, keeping
//      every tier of its own point in the lane's registers;
//   2. walks the adjoint down the region: its Lambda part first, taking the
//      adjoint of later regions just outside each tier from lambda slots,
//      then its V part, handing the 4 outermost values of each gap tier per
//      side on to the previous phase through the same slots.
// Slots are position-major [p][t & 1] with (w/2 + 2) positions per side, as
// in the forward engines: consumer left p = x + 2, right p = x - a; producer
// left p = x (x < a + 2), right p = x - a + 2 (x >= a - 2).
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <string>

#include "device_guard.h"
#include "internal.h"
#include "poison.h"
#include "swept.h"
#include "wave_tile.h"

namespace swept {
namespace ksadj {

constexpr int kW = 64;
constexpr int kS = 2;
constexpr int kH = kW / (2 * kS);  // 16 tiers (8 steps) per full triangle
constexpr int kA = kW / 2;         // inner seam
constexpr int kSL = kW + 2 * kS;
constexpr int kThreads = 256;
constexpr int kFwdPoints = 8;  // points per lane (and tiles per wave) of the checkpointing forward

// Coefficients of Jf(v)^T, formed on the host in FP64.
struct JtCoef {
  double i2dx;  // 1/(2 dx) = 2 (1/(4 dx)), so v i2dx rounds as (2 v) (1/(4 dx))
  double c1;    // idx2 - 4 idx4: the linear part of the w_{i-1}, w_{i+1} weights
  double c0;    // -(6 idx4 - 2 idx2): weight of w_i
  double c2;    // -idx4: weight of w_{i-2}, w_{i+2}
};

// (Jf(v)^T w)_i from v_i and w at i-2 .. i+2.
__device__ __forceinline__ double jt(double v, double wl2, double wl1, double w, double wr1, double wr2,
                                     const JtCoef& c) {
  const double s = v * c.i2dx;
  const double dm = -(s + c.c1);  // d f_{i-1} / d v_i
  const double dp = -(c.c1 - s);  // d f_{i+1} / d v_i
  return fmadd(c.c2, wr2, fmadd(c.c2, wl2, fmadd(c.c0, w, fmadd(dp, wr1, dm * wl1))));
}

using wave::lanes;
using wave::range_bits;

// The values two and one lanes to the left and right (zero past the wave).
struct Nb {
  double l2, l1, r1, r2;
};

__device__ __forceinline__ Nb nbrs(double v) {
  using wave::dpp_move0;
  Nb b;
  b.l1 = dpp_move0<wave::kDppWaveShr1>(v);
  b.r1 = dpp_move0<wave::kDppWaveShl1>(v);
  b.l2 = dpp_move0<wave::kDppWaveShr1>(b.l1);
  b.r2 = dpp_move0<wave::kDppWaveShl1>(b.r1);
  return b;
}

// Points -2, -1 and w, w+1 of a row that reaches past the tile.
__device__ __forceinline__ void fix_ends(Nb& b, double tl0, double tl1, double tr0, double tr1) {
  using wave::pick;
  b.l1 = pick(lanes(1ull), tl1, b.l1);
  b.l2 = pick(lanes(1ull), tl0, pick(lanes(2ull), tl1, b.l2));
  b.r1 = pick(lanes(1ull << (kW - 1)), tr0, b.r1);
  b.r2 = pick(lanes(1ull << (kW - 1)), tr1, pick(lanes(1ull << (kW - 2)), tr0, b.r2));
}

// Positions just outside Lambda tier t of a tile whose adjoint belongs to
// later regions: [2t - 4, 2t) and [w - 2t, w - 2t + 4).
__host__ __device__ constexpr uint64_t outside_bits(int t) {
  return range_bits(kS * t - 2 * kS, kS * t) | range_bits(kW - kS * t, kW - kS * t + 2 * kS);
}

// ---------------------------------------------------------------------------
// Checkpointing forward with P consecutive points per lane and P tiles of 64
// points per wave (64 / P lanes each).  It keeps no history beyond the last
// even tier, so a lane can hold several points: only the two outermost
// points on each side need lane shifts, and those serve P points.

// Lane mask of register r: the lanes whose point l P + r is set in `pos`
// (bit x = tile point x), in every tile of the wave.
template <int P>
__host__ __device__ constexpr uint64_t reg_bits(uint64_t pos, int r) {
  uint64_t m = 0;
  for (int l = 0; l < kW / P; ++l)
    if ((pos >> (l * P + r)) & 1)
      for (int tl = 0; tl < P; ++tl) m |= 1ull << (tl * (kW / P) + l);
  return m;
}

// Lanes holding the first (last) points of a tile.
template <int P>
__host__ __device__ constexpr uint64_t tile_end_bits(bool last) {
  uint64_t m = 0;
  for (int tl = 0; tl < P; ++tl) m |= 1ull << (tl * (kW / P) + (last ? kW / P - 1 : 0));
  return m;
}

// Points -2, -1 (lo) and P, P+1 (hi) around a lane's P points of a row.
struct Halo {
  double lo0, lo1, hi0, hi1;
};

template <int P>
__device__ __forceinline__ Halo halo(const double (&row)[P]) {
  using wave::dpp_move0;
  return Halo{dpp_move0<wave::kDppWaveShr1>(row[P - 2]), dpp_move0<wave::kDppWaveShr1>(row[P - 1]),
              dpp_move0<wave::kDppWaveShl1>(row[0]), dpp_move0<wave::kDppWaveShl1>(row[1])};
}

template <int P>
__device__ __forceinline__ double at(const double (&row)[P], const Halo& h, int i) {
  return i == -2 ? h.lo0 : (i == -1 ? h.lo1 : (i == P ? h.hi0 : (i == P + 1 ? h.hi1 : row[i])));
}

// Tier t+1 from tier t over a lane's points: the predictor (t+1 odd) or the
// final stage with u at the previous even tier `ue`.
template <int P, bool PRED>
__device__ __forceinline__ void fwd_tier(double (&row)[P], const double (&ue)[P], const Halo& h,
                                         const Consts<double>& k) {
  double nv[P];
#pragma unroll
  for (int r = 0; r < P; ++r) {
    if constexpr (PRED)
      nv[r] = ks_predictor(at<P>(row, h, r - 2), at<P>(row, h, r - 1), row[r], at<P>(row, h, r + 1),
                           at<P>(row, h, r + 2), k);
    else
      nv[r] = ks_final(ue[r], at<P>(row, h, r - 2), at<P>(row, h, r - 1), row[r], at<P>(row, h, r + 1),
                       at<P>(row, h, r + 2), k);
  }
#pragma unroll
  for (int r = 0; r < P; ++r) row[r] = nv[r];
}

// V tiers T .. h-1: insert the bands of tier T ([a-4-2T, a-2T) and
// [a+2T, a+2T+4)), keep u of the even tiers, compute tier T+1.  Tiers and
// registers are template arguments so every lane mask is a constant.
template <int P, int T, int R>
__device__ __forceinline__ void fwd_insert(double (&row)[P], const double (&bv0)[P], const double (&bv1)[P]) {
  if constexpr (R < P) {
    constexpr uint64_t m = reg_bits<P>(range_bits(kA - 2 * kS - kS * T, kA - kS * T) |
                                           range_bits(kA + kS * T, kA + kS * T + 2 * kS),
                                       R);
    if constexpr (m != 0) row[R] = wave::pick(lanes(m), (T & 1) ? bv1[R] : bv0[R], row[R]);
    fwd_insert<P, T, R + 1>(row, bv0, bv1);
  }
}

template <int P, int T>
__device__ __forceinline__ void fwd_v(double (&row)[P], double (&ue)[P], const double (&bv0)[P],
                                      const double (&bv1)[P], const Halo& tips, const Consts<double>& k) {
  if constexpr (T < kH) {
    fwd_insert<P, T, 0>(row, bv0, bv1);
    if constexpr ((T & 1) == 0) {
#pragma unroll
      for (int r = 0; r < P; ++r) ue[r] = row[r];
    }
    Halo h = halo<P>(row);
    if constexpr (T == kH - 1) {
      // points -2, -1 and w, w+1 of tier h-1 come from the slots
      const bool first = lanes(tile_end_bits<P>(false)), last = lanes(tile_end_bits<P>(true));
      h.lo0 = wave::pick(first, tips.lo0, h.lo0);
      h.lo1 = wave::pick(first, tips.lo1, h.lo1);
      h.hi0 = wave::pick(last, tips.hi0, h.hi0);
      h.hi1 = wave::pick(last, tips.hi1, h.hi1);
    }
    fwd_tier<P, ((T + 1) & 1) != 0>(row, ue, h, k);
    fwd_v<P, T + 1>(row, ue, bv0, bv1, tips, k);
  }
}

// Lambda tiers M .. h-1 (tier h + M of the region): compute tier M (M > 0),
// then store its bands, [2M, 2M+4) to the left slot (p = x) and
// [w-2M-4, w-2M) to the right slot (p = x - a + 2), from the lanes that own
// them, one entry per tier parity.
template <int P, int M, int R>
__device__ __forceinline__ void fwd_store(const double (&row)[P], double* outL, double* outR, bool valid) {
  if constexpr (R < P) {
    constexpr uint64_t ml = reg_bits<P>(range_bits(kS * M, kS * M + 2 * kS), R);
    constexpr uint64_t mr = reg_bits<P>(range_bits(kW - kS * M - 2 * kS, kW - kS * M), R);
    if constexpr (ml != 0) {
      if (valid && lanes(ml)) outL[2 * R + (M & 1)] = row[R];
    }
    if constexpr (mr != 0) {
      if (valid && lanes(mr)) outR[2 * R + (M & 1)] = row[R];
    }
    fwd_store<P, M, R + 1>(row, outL, outR, valid);
  }
}

template <int P, int M>
__device__ __forceinline__ void fwd_l(double (&row)[P], double (&ue)[P], double* outL, double* outR, bool valid,
                                      const Consts<double>& k) {
  if constexpr (M < kH) {
    if constexpr (M > 0) {
      const Halo h = halo<P>(row);
      fwd_tier<P, ((kH + M) & 1) != 0>(row, ue, h, k);
      if constexpr (((kH + M) & 1) == 0) {
#pragma unroll
        for (int r = 0; r < P; ++r) ue[r] = row[r];
      }
    }
    fwd_store<P, M, 0>(row, outL, outR, valid);
    fwd_l<P, M + 1>(row, ue, outL, outR, valid, k);
  }
}

template <int P, bool HV, bool HL>
__global__ void __launch_bounds__(kW)
forward_kernel(const double* __restrict__ ustart, double* __restrict__ uT, const double* __restrict__ ck_in,
               double* __restrict__ ck_out, Consts<double> k, int64_t n, int64_t nt, int p) {
  static_assert(P >= 2, "the lane shifts carry two points per side");
  constexpr int LPT = kW / P;  // lanes per tile
  const int lane = threadIdx.x;
  const int l = lane % LPT;
  const int64_t j = (int64_t)blockIdx.x * P + lane / LPT;  // tile
  const bool valid = j < nt;
  const int64_t jj = valid ? j : 0;  // tiles past the end read tile 0 and store nothing
  const int64_t b = blockIdx.y;
  const int par = p & 1;
  const int64_t origin = jj * kW + (par ? kA : 0);
  const int64_t base = b * 2 * nt * kSL;
  const int64_t sL = base + (par ? (nt + jj) * kSL : jj * kSL);
  const int64_t sR = base + (par ? (jj + 1 == nt ? 0 : jj + 1) * kSL : (nt + jj) * kSL);
  int64_t gidx[P];
#pragma unroll
  for (int r = 0; r < P; ++r) {
    int64_t gx = origin + l * P + r;
    if (gx >= n) gx -= n;
    gidx[r] = b * n + gx;
  }
  double row[P], ue[P];
  if constexpr (!HV) {
#pragma unroll
    for (int r = 0; r < P; ++r) row[r] = ustart[gidx[r]];
  } else {
    double bv0[P], bv1[P];
#pragma unroll
    for (int r = 0; r < P; ++r) {
      const int x = l * P + r;
      const int64_t src = x < kA ? sL + 2 * (x + kS) : sR + 2 * (x - kA);
      bv0[r] = ck_in[src];
      bv1[r] = ck_in[src + 1];
      row[r] = 0.0;
      ue[r] = 0.0;
    }
    // band points -2, -1, w, w+1 of tier h-1
    constexpr int tp = (kH - 1) & 1;
    const Halo tips{ck_in[sL + tp], ck_in[sL + 2 + tp], ck_in[sR + 2 * kA + tp], ck_in[sR + 2 * (kA + 1) + tp]};
    fwd_v<P, 0>(row, ue, bv0, bv1, tips, k);
  }
  if constexpr (HL) {
#pragma unroll
    for (int r = 0; r < P; ++r) ue[r] = row[r];  // tier h is even
    double* const outL = ck_out + sL + 2 * (l * P);
    double* const outR = ck_out + sR + 2 * (l * P - kA + kS);
    fwd_l<P, 0>(row, ue, outL, outR, valid, k);
  } else {
    if (valid) {
#pragma unroll
      for (int r = 0; r < P; ++r) uT[gidx[r]] = row[r];
    }
  }
}

// One swept region of one tile in one wave64 (lane x = tile point x).
// The fused reverse launch of one phase: recompute the region, then walk the
// adjoint down through it.  HV: the region has a V part (every phase but the
// first); HL: it has a Lambda part (every phase but the last).
template <bool HV, bool HL>
__global__ void __launch_bounds__(kW)
region_kernel(const double* __restrict__ ustart, const double* __restrict__ ck_in, const double* __restrict__ gT,
              double* lam_slots, double* __restrict__ g_ur, Consts<double> k, JtCoef c, int64_t n, int64_t nt,
              int p) {
  using wave::pick;
  const int x = threadIdx.x;
  const int64_t j = blockIdx.x;  // tile
  const int64_t b = blockIdx.y;  // grid of the batch
  const int par = p & 1;
  const int64_t origin = j * kW + (par ? kA : 0);
  const int64_t base = b * 2 * nt * kSL;
  const int64_t sL = base + (par ? (nt + j) * kSL : j * kSL);
  const int64_t sR = base + (par ? (j + 1 == nt ? 0 : j + 1) * kSL : (nt + j) * kSL);
  int64_t gx = origin + x;
  if (gx >= n) gx -= n;
  const int64_t gidx = b * n + gx;
  // this lane's entry in the incoming slots (one value per tier parity)
  const int64_t src = x < kA ? sL + 2 * (x + kS) : sR + 2 * (x - kA);
  // this lane's outgoing adjoint slot entries: left side p = x, right side
  // p = x - a + 2, one value per tier parity; a lane only stores where it
  // owns a band point
  double* const outL = lam_slots + sL + 2 * x;
  double* const outR = lam_slots + sR + 2 * (x - kA + kS);

  // ------------------------------------------------ forward recompute --
  double hist[2 * kH];  // u or q at (x, d), d = 0 .. 2h-1
  if constexpr (!HV) {
    hist[kH] = ustart[gidx];
  } else {
    const double bv0 = ck_in[src], bv1 = ck_in[src + 1];
    // band points -2, -1, w, w+1 of tier h-1
    constexpr int tp = (kH - 1) & 1;
    const double tl0 = ck_in[sL + tp], tl1 = ck_in[sL + 2 + tp];
    const double tr0 = ck_in[sR + 2 * kA + tp], tr1 = ck_in[sR + 2 * (kA + 1) + tp];
    double row = 0.0;
#pragma unroll
    for (int t = 0; t < kH; ++t) {
      // bands of tier t: [a-4-2t, a-2t) and [a+2t, a+2t+4)
      const uint64_t band = range_bits(kA - 2 * kS - kS * t, kA - kS * t) | range_bits(kA + kS * t, kA + kS * t + 2 * kS);
      row = pick(lanes(band), (t & 1) ? bv1 : bv0, row);
      hist[t] = row;
      Nb nb = nbrs(row);
      if (t == kH - 1) fix_ends(nb, tl0, tl1, tr0, tr1);
      if ((t + 1) & 1)
        row = ks_predictor(nb.l2, nb.l1, row, nb.r1, nb.r2, k);
      else
        row = ks_final(hist[t > 0 ? t - 1 : 0], nb.l2, nb.l1, row, nb.r1, nb.r2, k);
    }
    hist[kH] = row;
  }
  if constexpr (HL) {
    double row = hist[kH];
#pragma unroll
    for (int m = 0; m < kH; ++m) {
      if (m > 0) {
        const Nb nb = nbrs(row);
        if ((kH + m) & 1)
          row = ks_predictor(nb.l2, nb.l1, row, nb.r1, nb.r2, k);
        else
          row = ks_final(hist[kH + m - 2], nb.l2, nb.l1, row, nb.r1, nb.r2, k);
        hist[kH + m] = row;
      }
    }
  }
  {
    // --------------------------------------------------- adjoint sweep --
    double in0 = 0.0, in1 = 0.0, ll0 = 0.0, ll1 = 0.0, lr0 = 0.0, lr1 = 0.0;
    if constexpr (HL) {
      in0 = lam_slots[src];
      in1 = lam_slots[src + 1];
      // adjoint of points -2, -1, w, w+1 at tier h+1
      ll0 = lam_slots[sL + 1];
      ll1 = lam_slots[sL + 3];
      lr0 = lam_slots[sR + 2 * kA + 1];
      lr1 = lam_slots[sR + 2 * (kA + 1) + 1];
    }
    double lam = 0.0, lam2 = 0.0;  // adjoint at tiers d+1 and d+2
    if constexpr (HL)
      lam = pick(lanes(outside_bits(kH)), (kH & 1) ? in1 : in0, lam);
    else
      lam = gT[gidx];  // the region's top tier h is u_T
    double o0 = 0.0, o1 = 0.0;  // this lane's outgoing adjoint, by tier parity
#pragma unroll
    for (int d = HL ? 2 * kH - 1 : kH; d >= (HV ? 1 : kH); --d) {
      if (HL || d < kH) {
        Nb nb = nbrs(lam);
        if (HL && d == kH) fix_ends(nb, ll0, ll1, lr0, lr1);
        const double g = jt(hist[d], nb.l2, nb.l1, lam, nb.r1, nb.r2, c);
        const double nw = (d & 1) ? k.dt * g : fmadd(k.dth, g, lam2 + lam);
        lam2 = lam;
        lam = nw;
        if (HL && d > kH) {
          const int t = d - kH;
          lam = pick(lanes(outside_bits(t)), (t & 1) ? in1 : in0, lam);
        }
      }
      if (HV && d <= kH) {
        // the 4 outermost values on each side of gap(d) go to the previous phase
        // (lanes [a-2d, a-2d+4) and [a+2d-4, a+2d)).  A lane hands on at
        // most two tiers over both sides, of different parity (and the same
        // value where both sides take one tier), so one register per parity
        // collects them.
        const bool hand = lanes(range_bits(kA - kS * d, kA - kS * d + 2 * kS) |
                                range_bits(kA + kS * d - 2 * kS, kA + kS * d));
        if (d & 1)
          o1 = pick(hand, lam, o1);
        else
          o0 = pick(hand, lam, o0);
        // select here, not at the stores: deferred selects keep every tier's
        // adjoint and mask live
        asm volatile("" : "+v"(o0), "+v"(o1));
      }
      if (!HV && d == kH) g_ur[gidx] = lam;
    }
    if constexpr (HV) {
      // left: lanes x < a+2 at d = ceil((a-x)/2) + 0, 1; right: lanes
      // x >= a-2 at d = floor((x-a)/2) + 1, 2 (d in [1, h])
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        const int dl = (kA - x + 1) / 2 + e;
        if (x < kA + kS && dl >= 1 && dl <= kH) outL[dl & 1] = (dl & 1) ? o1 : o0;
        const int dr = (x - kA + 2) / 2 + e;
        if (x >= kA - kS && dr >= 1 && dr <= kH)
          outR[dr & 1] = (dr & 1) ? o1 : o0;
      }
    }
  }
}

// Periodic neighbour of x at offset o (|o| <= 2 < n).
__device__ __forceinline__ int64_t wrap(int64_t x, int o, int64_t n) {
  int64_t y = x + o;
  if (y < 0) y += n;
  if (y >= n) y -= n;
  return y;
}

// The predictor at x of the row v (period n).
__device__ __forceinline__ double pred_at(const double* v, int64_t x, int64_t n, const Consts<double>& k) {
  return ks_predictor(v[wrap(x, -2, n)], v[wrap(x, -1, n)], v[x], v[wrap(x, 1, n)], v[wrap(x, 2, n)], k);
}

// Leading classic steps, forward: q = u + (dt/2) f(u) ...
__global__ void __launch_bounds__(kThreads)
rem_pred_kernel(const double* __restrict__ u, double* __restrict__ q, Consts<double> k, int64_t n, int64_t total) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i >= total) return;
  const double* v = u + (i / n) * n;
  const int64_t x = i % n;
  q[i] = pred_at(v, x, n, k);
}

// ... then u' = u + dt f(q), out of place.
__global__ void __launch_bounds__(kThreads)
rem_final_kernel(const double* __restrict__ u, const double* __restrict__ q, double* __restrict__ un,
                 Consts<double> k, int64_t n, int64_t total) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i >= total) return;
  const double* w = q + (i / n) * n;
  const int64_t x = i % n;
  un[i] = ks_final(u[i], w[wrap(x, -2, n)], w[wrap(x, -1, n)], w[x], w[wrap(x, 1, n)], w[wrap(x, 2, n)], k);
}

// Leading classic steps, reverse: mu = dt Jf(q)^T lambda', with q at the
// own point recomputed from u ...
__global__ void __launch_bounds__(kThreads)
rem_mu_kernel(const double* __restrict__ u, const double* __restrict__ lin, double* __restrict__ mu,
              Consts<double> k, JtCoef c, int64_t n, int64_t total) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i >= total) return;
  const int64_t row = (i / n) * n;
  const int64_t x = i % n;
  const double* v = u + row;
  const double* l = lin + row;
  const double q = pred_at(v, x, n, k);
  mu[i] = k.dt * jt(q, l[wrap(x, -2, n)], l[wrap(x, -1, n)], l[x], l[wrap(x, 1, n)], l[wrap(x, 2, n)], c);
}

// ... then lambda = (lambda' + mu) + (dt/2) Jf(u)^T mu.
__global__ void __launch_bounds__(kThreads)
rem_lam_kernel(const double* __restrict__ u, const double* __restrict__ lin, const double* __restrict__ mu,
               double* __restrict__ lout, Consts<double> k, JtCoef c, int64_t n, int64_t total) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i >= total) return;
  const int64_t row = (i / n) * n;
  const int64_t x = i % n;
  const double* m = mu + row;
  const double g = jt(u[i], m[wrap(x, -2, n)], m[wrap(x, -1, n)], m[x], m[wrap(x, 1, n)], m[wrap(x, 2, n)], c);
  lout[i] = fmadd(k.dth, g, lin[i] + mu[i]);
}

}  // namespace ksadj
}  // namespace swept

struct swept_ks_adjoint_s {
  int32_t batch = 0;
  int64_t n = 0, steps = 0, nt = 0;
  int K = 0;  // full phases of 8 steps; phases 0..K
  int r = 0;  // leading classic steps
  swept::Consts<double> k{};
  swept::ksadj::JtCoef c{};
  int device = 0;  // current device at create: owns the buffers
  bool have_forward = false;
  bool poison = false;          // SWEPT_DEBUG_POISON: NaN-fill checkpoints and adjoint slots before use
  double* ckpt = nullptr;       // K phases x batch x 2nt x 68
  double* lam_slots = nullptr;  // batch x 2nt x 68
  double* rem = nullptr;        // (r+1) states x batch x n: u_0 .. u_r
  double* tmp = nullptr;        // batch x n: predictor / mu
  double* lam_a = nullptr;      // batch x n
  double* lam_b = nullptr;
  size_t ckpt_bytes = 0;
};

namespace {

using swept::ksadj::kSL;
using swept::ksadj::kThreads;
using swept::ksadj::kW;

int kfail(int code, const std::string& m) { return swept::set_error(code, m); }
int khip(hipError_t e, const char* what) {
  return kfail(SWEPT_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

void ks_free(swept_ks_adjoint_s* a) {
  for (double* q : {a->ckpt, a->lam_slots, a->rem, a->tmp, a->lam_a, a->lam_b})
    if (q) (void)hipFree(q);
  delete a;
}

dim3 grid_for(int64_t total) { return dim3((unsigned)((total + kThreads - 1) / kThreads)); }

}  // namespace

extern "C" {

int swept_ks_adjoint_create(swept_ks_adjoint* out, int32_t batch, int64_t n, int dtype, double dt, double dx,
                            int64_t steps) {
  if (!out) return kfail(SWEPT_EINVAL, "out must not be NULL");
  *out = nullptr;
  if (batch < 1 || batch > 65535) return kfail(SWEPT_EINVAL, "batch must be in [1, 65535]");
  if (dtype != SWEPT_F64) return kfail(SWEPT_EUNSUPPORTED, "the KS adjoint is built for SWEPT_F64");
  if (n < kW || n % kW != 0) return kfail(SWEPT_EUNSUPPORTED, "n must be a positive multiple of 64");
  if (steps < 1) return kfail(SWEPT_EINVAL, "steps must be >= 1");
  if (!std::isfinite(dt) || !std::isfinite(dx) || dx == 0.0)
    return kfail(SWEPT_EINVAL, "dt, dx must be finite, dx != 0");
  const int64_t total = (int64_t)batch * n;
  // the remainder steps launch one work-item per point of the batch
  if ((total + kThreads - 1) / kThreads * kThreads > (int64_t)UINT32_MAX)
    return kfail(SWEPT_EUNSUPPORTED, "batch x n exceeds one launch (2^32 - 1 work-items)");
  auto* a = new (std::nothrow) swept_ks_adjoint_s();
  if (!a) return kfail(SWEPT_ENOMEM, "host allocation failed");
  a->batch = batch;
  a->n = n;
  a->steps = steps;
  a->nt = n / kW;
  constexpr int spp = swept::ksadj::kH / 2;
  a->r = (int)(steps % spp);
  a->K = (int)(steps / spp);
  a->poison = swept::debug_poison_requested();
  // same formulas as swept_plan_create for SWEPT_KS_RK2 (Sec. 4.1, Sec. 5)
  a->k = swept::make_consts<double>(dt, dx, 0.0);
  a->c.i2dx = 2.0 * a->k.i4dx;
  a->c.c1 = a->k.idx2 - 4.0 * a->k.idx4;
  a->c.c0 = -(6.0 * a->k.idx4 - 2.0 * a->k.idx2);
  a->c.c2 = -a->k.idx4;
  const hipError_t de = hipGetDevice(&a->device);
  if (de != hipSuccess) {
    delete a;
    return khip(de, "hipGetDevice");
  }
  const size_t state = (size_t)total * sizeof(double);
  const size_t slots = (size_t)batch * 2 * (size_t)a->nt * kSL * sizeof(double);
  a->ckpt_bytes = (size_t)a->K * slots;
  struct Alloc {
    double** p;
    size_t bytes;
  } allocs[] = {
      {&a->ckpt, std::max<size_t>(a->ckpt_bytes, 8)},
      {&a->lam_slots, slots},
      {&a->rem, (size_t)(a->r + 1) * state},
      {&a->tmp, state},
      {&a->lam_a, state},
      {&a->lam_b, state},
  };
  for (const Alloc& al : allocs) {
    const hipError_t e = hipMalloc(reinterpret_cast<void**>(al.p), al.bytes);
    if (e != hipSuccess) {
      ks_free(a);
      return kfail(SWEPT_ENOMEM, std::string("hipMalloc(KS adjoint workspace): ") + hipGetErrorString(e));
    }
  }
  *out = a;
  return SWEPT_OK;
}

int swept_ks_forward_ckpt(swept_ks_adjoint a, const void* u0, void* uT, void* stream) {
  if (!a) return kfail(SWEPT_EINVAL, "KS adjoint plan must not be NULL");
  if (!u0 || !uT) return kfail(SWEPT_EINVAL, "u0 and uT must not be NULL");
  swept::DeviceGuard g(a->device);
  if (!g.ok) return khip(g.err, "hipSetDevice");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int64_t total = (int64_t)a->batch * a->n;
  const size_t state = (size_t)total * sizeof(double);
  hipError_t e = a->poison ? swept::poison_fill(a->ckpt, a->ckpt_bytes, 8, st) : hipSuccess;
  // leading classic steps: u_0 .. u_r kept for the reverse sweep
  if (e == hipSuccess) e = hipMemcpyAsync(a->rem, u0, state, hipMemcpyDeviceToDevice, st);
  for (int m = 0; m < a->r && e == hipSuccess; ++m) {
    const double* um = a->rem + (size_t)m * total;
    hipLaunchKernelGGL(swept::ksadj::rem_pred_kernel, grid_for(total), dim3(kThreads), 0, st, um, a->tmp, a->k,
                       a->n, total);
    e = hipGetLastError();
    if (e != hipSuccess) break;
    hipLaunchKernelGGL(swept::ksadj::rem_final_kernel, grid_for(total), dim3(kThreads), 0, st, um, a->tmp,
                       a->rem + (size_t)(m + 1) * total, a->k, a->n, total);
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
      constexpr int FP = swept::ksadj::kFwdPoints;
      auto kern = p == 0 ? swept::ksadj::forward_kernel<FP, false, true>
                         : (p == a->K ? swept::ksadj::forward_kernel<FP, true, false>
                                      : swept::ksadj::forward_kernel<FP, true, true>);
      hipLaunchKernelGGL(kern, dim3((unsigned)((a->nt + FP - 1) / FP), (unsigned)a->batch), dim3(kW), 0, st, ur,
                         static_cast<double*>(uT), ck_in, ck_out, a->k, a->n, a->nt, p);
      e = hipGetLastError();
    }
  }
  if (e != hipSuccess) return khip(e, "swept_ks_forward_ckpt");
  a->have_forward = true;
  return SWEPT_OK;
}

int swept_ks_adjoint_run(swept_ks_adjoint a, const void* g_uT, void* g_u0, void* stream) {
  if (!a) return kfail(SWEPT_EINVAL, "KS adjoint plan must not be NULL");
  if (!g_uT || !g_u0) return kfail(SWEPT_EINVAL, "g_uT and g_u0 must not be NULL");
  if (!a->have_forward) return kfail(SWEPT_EINVAL, "swept_ks_forward_ckpt must run first");
  swept::DeviceGuard g(a->device);
  if (!g.ok) return khip(g.err, "hipSetDevice");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int64_t total = (int64_t)a->batch * a->n;
  const size_t state = (size_t)total * sizeof(double);
  const size_t pslots = (size_t)a->batch * 2 * (size_t)a->nt * kSL;
  hipError_t e = a->poison ? swept::poison_fill(a->lam_slots, pslots * sizeof(double), 8, st) : hipSuccess;
  // adjoint at step r: from the swept sweep (or g_uT itself when T < 8)
  double* lam_r = a->r > 0 ? a->lam_a : static_cast<double*>(g_u0);
  if (a->K == 0) {
    e = hipMemcpyAsync(lam_r, g_uT, state, hipMemcpyDeviceToDevice, st);
  } else {
    const double* ur = a->rem + (size_t)a->r * total;
    for (int p = a->K; p >= 0 && e == hipSuccess; --p) {
      const double* ck_in = p > 0 ? a->ckpt + (size_t)(p - 1) * pslots : nullptr;
      auto kern = p == 0 ? swept::ksadj::region_kernel<false, true>
                         : (p == a->K ? swept::ksadj::region_kernel<true, false>
                                      : swept::ksadj::region_kernel<true, true>);
      hipLaunchKernelGGL(kern, dim3((unsigned)a->nt, (unsigned)a->batch), dim3(kW), 0, st, ur, ck_in,
                         static_cast<const double*>(g_uT), a->lam_slots, lam_r, a->k, a->c, a->n, a->nt, p);
      e = hipGetLastError();
    }
  }
  // leading classic steps backwards, m = r-1 .. 0
  double* lin = lam_r;
  for (int m = a->r - 1; m >= 0 && e == hipSuccess; --m) {
    const double* um = a->rem + (size_t)m * total;
    double* lout = m == 0 ? static_cast<double*>(g_u0) : (lin == a->lam_a ? a->lam_b : a->lam_a);
    hipLaunchKernelGGL(swept::ksadj::rem_mu_kernel, grid_for(total), dim3(kThreads), 0, st, um, lin, a->tmp, a->k,
                       a->c, a->n, total);
    e = hipGetLastError();
    if (e != hipSuccess) break;
    hipLaunchKernelGGL(swept::ksadj::rem_lam_kernel, grid_for(total), dim3(kThreads), 0, st, um, lin, a->tmp,
                       lout, a->k, a->c, a->n, total);
    e = hipGetLastError();
    lin = lout;
  }
  if (e != hipSuccess) return khip(e, "swept_ks_adjoint_run");
  return SWEPT_OK;
}

int swept_ks_adjoint_info(swept_ks_adjoint a, size_t* checkpoint_bytes, int* tile_width, int* steps_per_cycle,
                          int64_t* leading_classic_steps) {
  if (!a) return kfail(SWEPT_EINVAL, "KS adjoint plan must not be NULL");
  if (checkpoint_bytes) *checkpoint_bytes = a->ckpt_bytes;
  if (tile_width) *tile_width = kW;
  if (steps_per_cycle) *steps_per_cycle = swept::ksadj::kH / 2;
  if (leading_classic_steps) *leading_classic_steps = a->r;
  return SWEPT_OK;
}

void swept_ks_adjoint_destroy(swept_ks_adjoint a) {
  if (!a) return;
  swept::DeviceGuard g(a->device);
  ks_free(a);
}

}  // extern "C"
