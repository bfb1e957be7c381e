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
// Tiling.  Tiles of w = 64 points, one point per lane of one wave64, full
// (pure) phases of h = 32 steps; the T mod 32 leading steps run with the
// classic scheme and keep their states.  Forward: phase p writes its edge
// slots out of place, into checkpoint p.  Reverse, for p = K .. 0, one fused
// launch per phase: every tile
//   1. recomputes its forward region (V then Lambda) from checkpoint p-1,
//      keeping, for every tier, the Laplacian of the previous tier at its
//      own point in the lane's registers;
//   2. walks lambda down through the same region: its Lambda part first,
//      taking the lambda values of later regions just outside each tier from
//      lambda slots, then its V part, handing the two outermost values of each
//      gap tier on to the previous phase through the same slots;
//   3. adds lambda(x,t) (u(x-1,t-1) + u(x+1,t-1) - 2u(x,t-1)) over its points.
// The first phase (no V part) and the last (no Lambda part) run one region per
// wave (region_kernel); every other phase runs the chained launch
// (chain_kernel), where a wave keeps two regions of neighbouring tiles in
// flight on complementary lanes.
// The lambda slots mirror the forward edge slots: position-major [p][t & 1],
// (h+1) positions per side, updated in place by the tile that owns them.
// dJ/dalpha is summed per tile in phase order, then over tiles and remainder
// blocks in a fixed order: the result does not depend on scheduling.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <string>
#include <type_traits>
#include <vector>

#include "device_guard.h"
#include "internal.h"
#include "poison.h"
#include "swept.h"
#include "wave_tile.h"

namespace swept {
namespace adj {

constexpr int kW = 64;
constexpr int kH = 32;  // w / 2: tiers of a full triangle
constexpr int kA = 32;  // inner seam
constexpr int kSL = kW + 2;
constexpr int kRemThreads = 256;
constexpr int kFwdPoints = 8;  // points per lane (and tiles per wave) of the checkpointing forward

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

// Lanes computed at diamond tier d: the gap [a-d, a+d) in the V part
// (d <= h), [d-h, w-d+h) in the Lambda part.
__host__ __device__ constexpr uint64_t row_bits(int d) {
  return d <= kH ? wave::range_bits(kA - d, kA + d) : wave::range_bits(d - kH, kW - d + kH);
}

// Lanes [lo, lo + 2): the two points of an edge band.
__host__ __device__ constexpr uint64_t pair_bits(int lo) { return wave::range_bits(lo, lo + 2); }

// One swept region of one tile, held in one wave64: lane x owns tile point x
// and keeps the region's states u(x, d) in registers, tier by tier; the
// neighbours of a point come from DPP lane shifts and the edge bands enter
// and leave through per-lane registers, so there is no LDS and no barrier.
//
// The fused reverse launch of one phase: recompute the region, walk lambda
// down through it and add the dJ/dalpha terms.  HV: the region has a V part
// (every phase but the first); HL: it has a Lambda part (every phase but the
// last).  Slots are position-major [p][t & 1] as in the forward engines:
// consumer left input p = x + 1, right input p = x - a; producer left side
// p = x (x <= a), right side p = x - a + 1 (x >= a - 1).
template <bool HV, bool HL>
__global__ void __launch_bounds__(kW)
region_kernel(const double* __restrict__ ustart, const double* __restrict__ ck_in, const double* __restrict__ gT,
              double* lam_slots, double* __restrict__ g_ur, double* __restrict__ partial,
              const Consts<double>* __restrict__ kb, int64_t n, int64_t nt, int p) {
  using wave::dpp_move0;
  using wave::kDppWaveShl1;
  using wave::kDppWaveShr1;
  using wave::lanes;
  using wave::pick;
  const int x = threadIdx.x;
  const int64_t j = blockIdx.x;  // tile
  const int64_t b = blockIdx.y;  // grid of the batch
  const Consts<double> k = kb[b];
  const int par = p & 1;
  const int64_t origin = j * kW + (par ? kA : 0);
  const int64_t base = b * 2 * nt * kSL;
  const int64_t sL = base + (par ? (nt + j) * kSL : j * kSL);
  const int64_t sR = base + (par ? (j + 1 == nt ? 0 : j + 1) * kSL : (nt + j) * kSL);
  int64_t gx = origin + x;
  if (gx >= n) gx -= n;
  const int64_t gidx = b * n + gx;
  // this lane's outgoing lambda slot entries: left side p = x, right side
  // p = x - a + 1, one value per tier parity; a lane only stores where it
  // owns a band point
  double* const outL = lam_slots + sL + 2 * x;
  double* const outR = lam_slots + sR + 2 * (x - kA + 1);

  // ------------------------------------------------ forward recompute --
  // The recompute keeps, for every tier d of the region, the Laplacian term
  // of the dJ/dalpha sum at this lane's point, lap[d] = (u(x-1,d-1) +
  // u(x+1,d-1)) - 2 u(x,d-1), formed from the neighbour sum the update uses.
  // Only dJ/dalpha reads it, a sum that matches the reference to rounding
  // rather than bit for bit, so it and the sum's terms use fused
  // multiply-adds of their own; lambda and dJ/du0 keep the update order of
  // heat_update.
  double lap[2 * kH];
  double top = 0.0;  // the region's row at tier h
  double tipL = 0.0, tipR = 0.0;  // points -1 and w at tier h-1
  if constexpr (!HV) {
    top = ustart[gidx];
  } else {
    // this lane's incoming band values, one per tier parity
    const int64_t src = x < kA ? sL + 2 * (x + 1) : sR + 2 * (x - kA);
    const double bv0 = ck_in[src], bv1 = ck_in[src + 1];
    tipL = ck_in[sL + ((kH - 1) & 1)];
    tipR = ck_in[sR + 2 * (kW - kA) + ((kH - 1) & 1)];
    double row = 0.0;
#pragma unroll
    for (int t = 0; t < kH; ++t) {
      // band of tier t: [a-t-2, a-t) and [a+t, a+t+2)
      row = pick(lanes(pair_bits(kA - t - 2) | pair_bits(kA + t)), (t & 1) ? bv1 : bv0, row);
      double lo = dpp_move0<kDppWaveShr1>(row), hi = dpp_move0<kDppWaveShl1>(row);
      if (t == kH - 1) {
        lo = pick(lanes(1ull), tipL, lo);
        hi = pick(lanes(1ull << (kW - 1)), tipR, hi);
      }
      const double sum = hi + lo;
      lap[t + 1] = __builtin_fma(-2.0, row, sum);
      row = fmadd(k.fo, sum, k.c * row);  // heat_update(lo, row, hi)
    }
    top = row;
  }
  if constexpr (HL) {
    double row = top;
#pragma unroll
    for (int m = 1; m < kH; ++m) {
      const double lo = dpp_move0<kDppWaveShr1>(row), hi = dpp_move0<kDppWaveShl1>(row);
      const double sum = hi + lo;
      lap[kH + m] = __builtin_fma(-2.0, row, sum);
      row = fmadd(k.fo, sum, k.c * row);  // heat_update(lo, row, hi)
    }
  }
  {
    // --------------------------------------------------- adjoint sweep --
    // lambda of later regions just outside Lambda tier h+m (m = 1 .. h):
    // [m-2, m) from the left slot (p = pos + 1), [w-m, w-m+2) from the right
    // (p = pos - (w - h)); one value per tier parity for every lane, and the
    // two points beyond the tile ends at m = 1.
    double in0 = 0.0, in1 = 0.0, ltipL = 0.0, ltipR = 0.0;
    if constexpr (HL) {
      const int64_t src = x < kW - kH ? sL + 2 * (x + 1) : sR + 2 * (x - (kW - kH));
      in0 = lam_slots[src];
      in1 = lam_slots[src + 1];
      ltipL = lam_slots[sL + 1];
      ltipR = lam_slots[sR + 2 * kH + 1];
    }
    double lam = 0.0, acc = 0.0;
    double o0 = 0.0, o1 = 0.0;  // this lane's outgoing lambda, by tier parity
    if constexpr (HL)
      lam = pick(lanes(pair_bits(kH - 2) | pair_bits(kW - kH)), (kH & 1) ? in1 : in0, lam);
    else
      lam = gT[gidx];  // lambda at the region's top tier h
#pragma unroll
    for (int d = HL ? 2 * kH - 1 : kH; d >= (HV ? 1 : kH); --d) {
      if (HL || d < kH) {  // lambda at tier d from tier d+1
        double lo = dpp_move0<kDppWaveShr1>(lam), hi = dpp_move0<kDppWaveShl1>(lam);
        if (HL && d == kH) {
          lo = pick(lanes(1ull), ltipL, lo);
          hi = pick(lanes(1ull << (kW - 1)), ltipR, hi);
        }
        lam = heat_update(lo, lam, hi, k);
      }
      if (HV || d != kH) {  // dJ/dalpha term lambda(x,d) (L u)(x, d-1)
        acc = pick(lanes(row_bits(d)), __builtin_fma(lam, lap[d], acc), acc);
        // settle this tier's sum here so that no term waits in a register
        asm volatile("" : "+v"(acc));
      }
      if (HV && d <= kH) {
        // the two outermost values on each side of gap(d) go to the previous
        // phase.  A lane hands on at most two tiers over both sides, of
        // different parity (and the same lambda where both sides take one
        // tier), so one register per parity collects them.
        const bool hand = lanes(pair_bits(kA - d) | pair_bits(kA + d - 2));
        if (d & 1)
          o1 = pick(hand, lam, o1);
        else
          o0 = pick(hand, lam, o0);
        // select here, not at the stores: deferred selects keep every tier's
        // lambda and mask live
        asm volatile("" : "+v"(o0), "+v"(o1));
      }
      if (!HV && d == kH) g_ur[gidx] = lam;
      if (HL && d > kH) {
        const int m = d - kH;
        lam = pick(lanes(pair_bits(m - 2) | pair_bits(kW - m)), (m & 1) ? in1 : in0, lam);
      }
    }
    if constexpr (HV) {
      // left side p = x: lanes x <= a at d = a-x, a-x+1; right side
      // p = x-a+1: lanes x >= a-1 at d = x-a+1, x-a+2 (d in [1, h])
      if (x <= kA) {
        const int d0 = kA - x, d1 = kA - x + 1;
        if (d0 >= 1) outL[d0 & 1] = (d0 & 1) ? o1 : o0;
        if (d1 <= kH) outL[d1 & 1] = (d1 & 1) ? o1 : o0;
      }
      if (x >= kA - 1) {
        const int d0 = x - kA + 1, d1 = x - kA + 2;
        if (d0 >= 1) outR[d0 & 1] = (d0 & 1) ? o1 : o0;
        if (d1 <= kH) outR[d1 & 1] = (d1 & 1) ? o1 : o0;
      }
    }
    // per-tile sum in a fixed order (x += x + s, s = 32 .. 1), added to this
    // tile's running sum
#pragma unroll
    for (int s = kW / 2; s > 0; s >>= 1) acc = acc + __shfl_down(acc, s, kW);
    if (x == 0) partial[b * nt + j] += acc;
  }
}

// ------------------------------------------------------------------------
// Chained reverse launch (every phase with both a V and a Lambda part).
//
// Within one region the V part widens tier by tier from the seam and the
// Lambda part narrows towards the top, so a wave that walks one region at a
// time leaves half of its lanes idle at every tier.  Here one wave walks a
// chain of consecutive tiles of one grid and keeps two regions in flight:
//   A_i: the forward recompute of the V part of tile i together with the
//        Lambda part of tile i-1;
//   B_i: the lambda walk of the Lambda part of tile i together with the V
//        part of tile i-1.
// Consecutive tiles of the chain use layouts rotated by 32 lanes against
// each other (tile point q in lane q for even chain positions, in lane
// (q + 32) mod 64 for odd ones), so a V part (centred on the seam, point 32)
// and a Lambda part (centred on the tile middle) of neighbouring positions
// fall on complementary lanes.  Lane shifts rotate across the wave, which
// joins points 31 and 32 of a rotated tile; the tile ends (points 0 and 63)
// take their outside neighbours from the tip registers as before.
//
// The Lambda part of A_i runs two tiers behind the V part's mirror tier
// (Lambda tier h+s+2 beside V tier s), and likewise in B_i (Lambda tier
// h+d+2 beside V tier d).  The four lanes that then belong to neither part
// are exactly those that hold the band values (A) or the injected lambda
// values of later regions (B), so each lane either computes a point of one
// of the two regions or holds an input of the next tier.
//
// For heat, lambda does not depend on u, so the two history sets a tile needs
// are made in either order: the lambda walk of tile i's Lambda part (B_i)
// keeps lambda per tier, the recompute of that part (A_{i+1}) pairs it with
// the Laplacian as it forms; the recompute of tile i's V part (A_i) keeps the
// Laplacian per tier, the lambda walk of that part (B_{i+1}) pairs it with
// lambda as it forms.  Register set Z[t] of one chain parity holds the V
// Laplacian of tier t on the V lanes and the Lambda lambda of tier h+t on
// the others; a slot is rewritten only two tiers after its last read.  The
// lambda values, the hand-off values and the edge slots are those of the
// one-region kernel bit for bit; the dJ/dalpha terms are the same products,
// summed per tile in another (fixed) order.
constexpr int kDppWaveRor1 = 0x13C;  // lane i <- lane i-1, lane 0 <- lane 63
constexpr int kDppWaveRol1 = 0x134;  // lane i <- lane i+1, lane 63 <- lane 0

// Lane mask of a set of tile points (bit q = point q) in layout L.
template <int L>
__host__ __device__ constexpr uint64_t lmask(uint64_t pts) {
  return L ? (pts << 32) | (pts >> 32) : pts;
}
// The lane of tile point q, and the point held by lane x, in layout L (the
// rotation by 32 is its own inverse).
template <int L>
__host__ __device__ constexpr int rot_lane(int q) {
  return L ? (q + 32) & 63 : q;
}

// Calls f(integral_constant<int, I>) for I = B, B+S, ... up to and including
// E, so that every step of a walk sees its tier as a constant expression.
template <int B, int E, int S, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr ((S > 0 && B <= E) || (S < 0 && B >= E)) {
    f(std::integral_constant<int, B>{});
    static_for<B + S, E, S>(f);
  }
}

// Lane masks of the chained walks, by layout L, step and use: a constant
// table read with scalar loads.  (A 64-bit mask has no literal form; formed
// from immediates in the loop, or kept in scalar registers across it, the
// masks cost more issue slots than the selects they drive.)
enum ChainMask { kCmBand, kCmAccA, kCmTipA0, kCmTipA1, kCmAccB, kCmHand, kCmInj, kCmTipB0, kCmTipB1, kCmKinds };
constexpr int kCmSteps = kH + 3;  // steps s = -1 .. h of A and d = h .. -1 of B
struct ChainMasks {
  uint64_t m[2][kCmSteps][kCmKinds];
};

__host__ __device__ constexpr uint64_t lmask_rt(int L, uint64_t pts) { return L ? (pts << 32) | (pts >> 32) : pts; }
__host__ __device__ constexpr int rot_lane_rt(int L, int q) { return L ? (q + 32) & 63 : q; }

constexpr ChainMasks make_chain_masks() {
  ChainMasks t{};
  for (int L = 0; L < 2; ++L) {
    for (int s = -1; s <= kH; ++s) {  // A: V tier s (layout L), Lambda tier h+s+2 (layout 1-L)
      uint64_t* e = t.m[L][s + 1];
      const int m = s + 2;
      e[kCmBand] = s >= 1 ? lmask_rt(L, pair_bits(kA - s - 1) | pair_bits(kA + s - 1)) : 0;
      e[kCmAccA] = m >= 1 && m <= kH - 1 ? lmask_rt(1 - L, wave::range_bits(m, kW - m)) : 0;
      e[kCmTipA0] = s == kH ? 1ull << rot_lane_rt(L, 0) : 0;
      e[kCmTipA1] = s == kH ? 1ull << rot_lane_rt(L, kW - 1) : 0;
    }
    for (int d = kH; d >= -1; --d) {  // B: V tier d (layout 1-L), Lambda tier h+d+2 (layout L)
      uint64_t* e = t.m[L][kH - d];
      const int m = d + 2;
      e[kCmAccB] = d >= 1 ? lmask_rt(1 - L, wave::range_bits(kA - d, kA + d)) : 0;
      e[kCmHand] = d >= 1 ? lmask_rt(1 - L, pair_bits(kA - d) | pair_bits(kA + d - 2)) : 0;
      e[kCmInj] = m >= 1 && m <= kH ? lmask_rt(L, pair_bits(m - 2) | pair_bits(kW - m)) : 0;
      e[kCmTipB0] = d == kH ? 1ull << rot_lane_rt(1 - L, 0) : 0;
      e[kCmTipB1] = d == kH ? 1ull << rot_lane_rt(1 - L, kW - 1) : 0;
    }
  }
  return t;
}
__constant__ ChainMasks kChainMasks = make_chain_masks();
typedef const __attribute__((address_space(4))) uint64_t* MaskPtr;

// dst = v on the lanes of m (a per-lane select).
__device__ __forceinline__ void set_on(uint64_t m, double v, double& dst) { dst = wave::pick(wave::lanes(m), v, dst); }

// acc = fma(a, b, acc) on the lanes of m, under an execution mask: one
// operation instead of a multiply-add and a select.  The empty asm statement
// cannot be speculated, so the block is not turned into a select; free of
// side effects, it lets the scheduler move loads across it.
__device__ __forceinline__ void fma_on(uint64_t m, double a, double b, double& acc) {
  if (wave::lanes(m)) {
    acc = __builtin_fma(a, b, acc);
    asm("" : "+v"(acc));
  }
}

// History writes in place: the new value takes the register of the slot's
// previous value (dead by then), which the register allocator does not find
// by itself across the chain loop.  Same operations and rounding as
// fma(-2, row, sum) and fma(a, b, c).
__device__ __forceinline__ void lap_into(double& z, double row, double sum) {
  asm("v_fma_f64 %0, -2.0, %1, %2" : "+v"(z) : "v"(row), "v"(sum));
}
__device__ __forceinline__ void fma_into(double& z, double a, double b, double c) {
  asm("v_fma_f64 %0, %1, %2, %3" : "+v"(z) : "v"(a), "v"(b), "v"(c));
}

// Chain position i (layout L = i mod 2): A_i then B_i, then the hand-off
// stores and the dJ/dalpha partial of tile i-1.  ZA is the register set of
// parity i, ZB that of parity i+1.
// Offsets of the slot entries that the lane holding tile point q of tile j
// reads: its band (or lambda) pair, and the outside neighbour of a tile end
// (point -1 for point 0, point w for point w-1; position 0 of the left slot,
// position w-a = h of the right one, odd tier parity).
__device__ __forceinline__ void tile_src(int64_t base, int64_t nt, int par, int64_t j, int q, int64_t& src,
                                         int64_t& tsrc) {
  const int64_t sL = base + (par ? (nt + j) * kSL : j * kSL);
  const int64_t sR = base + (par ? (j + 1 == nt ? 0 : j + 1) * kSL : (nt + j) * kSL);
  src = q < kA ? sL + 2 * (q + 1) : sR + 2 * (q - kA);
  tsrc = q == 0 ? sL + ((kH - 1) & 1) : sR + 2 * (kW - kA) + ((kH - 1) & 1);
}

// One tile's inputs staged in LDS by direct loads from global memory, a chain
// position ahead of their use, so that their latency is hidden without
// holding registers: per lane (layout of the tile), the band pair and the
// lambda pair of its point, and the slot position that holds the outside
// neighbour of a tile end (its odd-parity entry is the tip).
struct ChainStage {
  double band[kW][2];
  double lam[kW][2];
  double tip[kW][2];
  double ltip[kW][2];
};
typedef __attribute__((address_space(3))) void* LdsPtr;
constexpr int kWaitVmcnt0 = 0x0F70;  // s_waitcnt vmcnt(0), other counters not waited on

template <int L>
__device__ __forceinline__ void stage_tile(const double* ck_in, const double* lam_slots, int64_t base, int64_t nt,
                                           int par, int64_t j, int x, ChainStage& st) {
  int64_t src, tsrc;
  tile_src(base, nt, par, j, rot_lane<L>(x), src, tsrc);
  // lane x's 16 bytes land at byte 16x of the destination (tsrc is the odd
  // entry of its position: the pair starts one entry before)
  __builtin_amdgcn_global_load_lds(ck_in + src, (LdsPtr)&st.band[0][0], 16, 0, 0);
  __builtin_amdgcn_global_load_lds(lam_slots + src, (LdsPtr)&st.lam[0][0], 16, 0, 0);
  __builtin_amdgcn_global_load_lds(ck_in + tsrc - 1, (LdsPtr)&st.tip[0][0], 16, 0, 0);
  __builtin_amdgcn_global_load_lds(lam_slots + tsrc - 1, (LdsPtr)&st.ltip[0][0], 16, 0, 0);
}

// The outputs of tile j (layout L): the lambda values handed to the previous
// phase (o0, o1: by tier parity) and its running dJ/dalpha sum (lane 0).
// Left side p = q: points q <= a at d = a-q, a-q+1; right side p = q-a+1:
// points q >= a-1 at d = q-a+1, q-a+2 (d in [1, h]).  The two tiers of a
// lane differ in parity, so a lane with both in range fills both entries of
// its position, [p][0] = o0 and [p][1] = o1, with one 16-byte store: points
// 1 .. a-1 on the left, a .. w-2 on the right.  The four others have one
// tier each: point 0 left [0][0] and point w-1 right [h][0] (o0), point a-1
// right [0][1] and point a left [h][1] (o1).
template <int L>
__device__ __forceinline__ void store_outputs(double* lam_slots, double* __restrict__ partial, int64_t base,
                                              int64_t nt, int par, int64_t b, int64_t j, int x, double o0, double o1,
                                              double sum) {
  const int64_t sL = base + (par ? (nt + j) * kSL : j * kSL);
  const int64_t sR = base + (par ? (j + 1 == nt ? 0 : j + 1) * kSL : (nt + j) * kSL);
  const int q = rot_lane<L>(x);
  if (q >= 1 && q <= kW - 2) {
    double* const pos = lam_slots + (q < kA ? sL + 2 * q : sR + 2 * (q - kA + 1));
    *reinterpret_cast<double2*>(pos) = make_double2(o0, o1);
  }
  if (q == 0 || q == kA - 1 || q == kA || q == kW - 1) {
    double* const e = lam_slots + (q == 0 ? sL : (q == kA - 1 ? sR + 1 : (q == kA ? sL + 2 * kA + 1 : sR + 2 * kH)));
    *e = (q == 0 || q == kW - 1) ? o0 : o1;
  }
  if (x == 0) partial[b * nt + j] = sum;
}

template <int L>
__device__ __forceinline__ void chain_position(const double* __restrict__ ck_in, double* lam_slots,
                                               double* __restrict__ partial, const Consts<double>& k, int64_t b,
                                               int64_t nt, int par, int64_t j0, int64_t i, int64_t count, double& row,
                                               double& lam, double& ltp, double (&ZA)[kH + 1],
                                               double (&ZB)[kH + 1], ChainStage (&stage)[2], double& po0,
                                               double& po1, double& psum) {
  using wave::dpp_move0;
  // the lane index, opaque to the compiler in each position: lane-dependent
  // offsets are then formed where they are used instead of being kept (and
  // spilled) across the chain loop
  int x = threadIdx.x;
  asm volatile("" : "+v"(x));
  const int64_t base = b * 2 * nt * kSL;
  // the mask table of layout L; the empty asm statement keeps its loads in the
  // chain loop
  MaskPtr mt = (MaskPtr)(&kChainMasks.m[L][0][0]);
  asm volatile("" : "+s"(mt));
  // inputs of tile i from its stage (for i = count the stage holds the
  // finite inputs of an earlier tile, which only reach lanes whose results are
  // not kept): band values and tips of its V part here, lambda of later
  // regions beside its Lambda part and beyond its ends at the start of B_i;
  // then the inputs of tile i+1 are staged
  // (the stage was filled a position ago; waiting for every vector memory
  // operation here also covers the outputs stored at the start of that
  // position, long complete)
  __builtin_amdgcn_s_waitcnt(kWaitVmcnt0);
  const double bv0 = stage[L].band[x][0], bv1 = stage[L].band[x][1], tip = stage[L].tip[x][1];
  if (i + 1 < count) stage_tile<1 - L>(ck_in, lam_slots, base, nt, par, j0 + i + 1, x, stage[1 - L]);
  // outputs of tile i-2 (same layout), kept from the end of the last position
  if (i >= 2) store_outputs<L>(lam_slots, partial, base, nt, par, b, j0 + i - 2, x, po0, po1, psum);

  // ---- A_i: V tier s of tile i (layout L) beside Lambda tier h+s+2 of tile
  // i-1 (layout 1-L)
  double acc = 0.0;
  // masks of step index k are loaded two steps ahead of their use
  uint64_t ma[kCmSteps][2];
  static_for<0, 1, 1>([&](auto kc) {
    constexpr int kk = decltype(kc)::value;
    ma[kk][0] = mt[kk * kCmKinds + kCmBand];
    ma[kk][1] = mt[kk * kCmKinds + kCmAccA];
  });
  static_for<-1, kH, 1>([&](auto sc) {
    constexpr int s = decltype(sc)::value;
    if constexpr (s + 3 < kCmSteps) {
      ma[s + 3][0] = mt[(s + 3) * kCmKinds + kCmBand];
      ma[s + 3][1] = mt[(s + 3) * kCmKinds + kCmAccA];
    }
    if constexpr (s >= 1)  // band of tier s-1: [a-s-1, a-s+1) and [a+s-1, a+s+1)
      set_on(ma[s + 1][0], ((s - 1) & 1) ? bv1 : bv0, row);
    double lo = dpp_move0<kDppWaveRor1>(row), hi = dpp_move0<kDppWaveRol1>(row);
    if constexpr (s == kH) {
      set_on(mt[(s + 1) * kCmKinds + kCmTipA0], tip, lo);
      set_on(mt[(s + 1) * kCmKinds + kCmTipA1], tip, hi);
    }
    const double sum = hi + lo;
    double lap;
    if constexpr (s >= 1) {
      lap_into(ZA[s], row, sum);
      lap = ZA[s];
    } else {
      lap = __builtin_fma(-2.0, row, sum);
    }
    constexpr int m = s + 2;
    if constexpr (m >= 1 && m <= kH - 1)  // Lambda tier h+m of tile i-1: [m, w-m)
      fma_on(ma[s + 1][1], ZA[m], lap, acc);
    row = fmadd(k.fo, sum, k.c * row);  // heat_update(lo, row, hi)
  });

  // ---- B_i: Lambda tier h+d+2 of tile i (layout L) beside V tier d of tile
  // i-1 (layout 1-L), d = h .. -1
  const double in0 = stage[L].lam[x][0], in1 = stage[L].lam[x][1], ltn = stage[L].ltip[x][1];
  // the running dJ/dalpha sum of tile i-1, a walk ahead of its update
  double part = 0.0;
  if (i >= 1 && x == 0) part = partial[b * nt + j0 + i - 1];
  double o0 = 0.0, o1 = 0.0;
  uint64_t mb[kCmSteps][3];
  static_for<0, 1, 1>([&](auto kc) {
    constexpr int kk = decltype(kc)::value;
    mb[kk][0] = mt[kk * kCmKinds + kCmAccB];
    mb[kk][1] = mt[kk * kCmKinds + kCmHand];
    mb[kk][2] = mt[kk * kCmKinds + kCmInj];
  });
  static_for<kH, -1, -1>([&](auto dc) {
    constexpr int d = decltype(dc)::value;
    if constexpr (kH - d + 2 < kCmSteps) {
      mb[kH - d + 2][0] = mt[(kH - d + 2) * kCmKinds + kCmAccB];
      mb[kH - d + 2][1] = mt[(kH - d + 2) * kCmKinds + kCmHand];
      mb[kH - d + 2][2] = mt[(kH - d + 2) * kCmKinds + kCmInj];
    }
    double lo = dpp_move0<kDppWaveRor1>(lam), hi = dpp_move0<kDppWaveRol1>(lam);
    if constexpr (d == kH) {
      set_on(mt[(kH - d) * kCmKinds + kCmTipB0], ltp, lo);
      set_on(mt[(kH - d) * kCmKinds + kCmTipB1], ltp, hi);
    }
    constexpr int m = d + 2;
    // heat_update(lo, lam, hi); Lambda tier h+m of tile i is kept for A_{i+1}
    const double sum = hi + lo, t1 = k.c * lam;
    if constexpr (m >= 1 && m <= kH - 1) {
      fma_into(ZB[m], k.fo, sum, t1);
      lam = ZB[m];
    } else {
      lam = fmadd(k.fo, sum, t1);
    }
    if constexpr (d >= 1) {
      // dJ/dalpha term of V tier d of tile i-1, gap [a-d, a+d)
      fma_on(mb[kH - d][0], lam, ZB[d], acc);
      // the two outermost values on each side of the gap go to the previous
      // phase (one register per tier parity, as in the one-region kernel)
      const uint64_t hand = mb[kH - d][1];
      if constexpr (d & 1)
        set_on(hand, lam, o1);
      else
        set_on(hand, lam, o0);
      asm("" : "+v"(o0), "+v"(o1));
    }
    if constexpr (m >= 1 && m <= kH)  // lambda of later regions just outside Lambda tier h+m
      set_on(mb[kH - d][2], (m & 1) ? in1 : in0, lam);
  });


  if (i >= 1) {
    // outputs of tile i-1, stored at the start of the next position
#pragma unroll
    for (int s = kW / 2; s > 0; s >>= 1) acc = acc + __shfl_down(acc, s, kW);
    po0 = o0;
    po1 = o1;
    psum = part + acc;
  }
  ltp = ltn;
}

// The chained reverse launch of one middle phase: workgroup (c, b) walks
// tiles c*chain .. c*chain+chain-1 of grid b (fewer at the end of the grid).
// Measured on 64 grids of 2^18 points: chains of 8, 16 and 32 tiles take
// 0.458, 0.439 and 0.443 ms per launch (the first and last position of a
// chain carry one region each; long chains leave the last round of
// workgroups part-empty).
constexpr int kChain = 16;
__global__ void __launch_bounds__(kW) __attribute__((amdgpu_waves_per_eu(3)))
chain_kernel(const double* __restrict__ ck_in, double* lam_slots, double* __restrict__ partial,
             const Consts<double>* __restrict__ kb, int64_t nt, int p, int chain) {
  const int64_t b = blockIdx.y;
  const int64_t j0 = (int64_t)blockIdx.x * chain;
  const int64_t count = nt - j0 < chain ? nt - j0 : chain;
  const Consts<double> k = kb[b];
  const int par = p & 1;
  double Z0[kH + 1], Z1[kH + 1];
#pragma unroll
  for (int u = 0; u <= kH; ++u) Z0[u] = Z1[u] = 0.0;
  __shared__ ChainStage stage[2];
  const int64_t base = b * 2 * nt * kSL;
  stage_tile<0>(ck_in, lam_slots, base, nt, par, j0, threadIdx.x, stage[0]);
  double row = 0.0, lam = 0.0, ltp = 0.0, po0 = 0.0, po1 = 0.0, psum = 0.0;
  for (int64_t i = 0; i <= count; i += 2) {
    chain_position<0>(ck_in, lam_slots, partial, k, b, nt, par, j0, i, count, row, lam, ltp, Z0, Z1, stage, po0,
                          po1, psum);
    if (i + 1 > count) break;
    chain_position<1>(ck_in, lam_slots, partial, k, b, nt, par, j0, i + 1, count, row, lam, ltp, Z1, Z0, stage,
                          po0, po1, psum);
  }
  // the outputs of the last tile of the chain
  const int64_t jl = j0 + count - 1;
  if ((count - 1) & 1)
    store_outputs<1>(lam_slots, partial, base, nt, par, b, jl, threadIdx.x, po0, po1, psum);
  else
    store_outputs<0>(lam_slots, partial, base, nt, par, b, jl, threadIdx.x, po0, po1, psum);
}

// Lane mask of register r when each lane holds P consecutive tile points and
// a wave holds P tiles of 64 / P lanes: the lanes whose point l P + r is set
// in `pos` (bit x = tile point x), in every tile of the wave.
template <int P>
__host__ __device__ constexpr uint64_t reg_bits(uint64_t pos, int r) {
  uint64_t m = 0;
  for (int l = 0; l < kW / P; ++l)
    if ((pos >> (l * P + r)) & 1)
      for (int tl = 0; tl < P; ++tl) m |= 1ull << (tl * (kW / P) + l);
  return m;
}

// Lanes holding the first (last) point of a tile.
template <int P>
__host__ __device__ constexpr uint64_t tile_end_bits(bool last) {
  uint64_t m = 0;
  for (int tl = 0; tl < P; ++tl) m |= 1ull << (tl * (kW / P) + (last ? kW / P - 1 : 0));
  return m;
}

// One heat tier over a lane's P points; lo and hi are the neighbours of its
// first and last point.
template <int P>
__device__ __forceinline__ void fwd_update(double (&row)[P], double lo, double hi, const Consts<double>& k) {
  double prev = lo;
#pragma unroll
  for (int r = 0; r < P; ++r) {
    const double nv = heat_update(prev, row[r], r + 1 < P ? row[r + 1] : hi, k);
    prev = row[r];
    row[r] = nv;
  }
}

// V tiers T .. h-1 of the forward: insert the band values of tier T
// ([a-T-2, a-T) and [a+T, a+T+2)) into the registers that hold them, then
// compute tier T+1.  Tiers and registers are template arguments so that
// every lane mask is a compile-time constant.
template <int P, int T, int R>
__device__ __forceinline__ void fwd_insert(double (&row)[P], const double (&bv0)[P], const double (&bv1)[P]) {
  if constexpr (R < P) {
    constexpr uint64_t m = reg_bits<P>(pair_bits(kA - T - 2) | pair_bits(kA + T), R);
    if constexpr (m != 0) row[R] = wave::pick(wave::lanes(m), (T & 1) ? bv1[R] : bv0[R], row[R]);
    fwd_insert<P, T, R + 1>(row, bv0, bv1);
  }
}

template <int P, int T>
__device__ __forceinline__ void fwd_v(double (&row)[P], const double (&bv0)[P], const double (&bv1)[P], double tipL,
                                      double tipR, const Consts<double>& k) {
  if constexpr (T < kH) {
    fwd_insert<P, T, 0>(row, bv0, bv1);
    double lo = wave::dpp_move0<wave::kDppWaveShr1>(row[P - 1]);
    double hi = wave::dpp_move0<wave::kDppWaveShl1>(row[0]);
    if constexpr (T == kH - 1) {
      lo = wave::pick(wave::lanes(tile_end_bits<P>(false)), tipL, lo);
      hi = wave::pick(wave::lanes(tile_end_bits<P>(true)), tipR, hi);
    }
    fwd_update<P>(row, lo, hi, k);
    fwd_v<P, T + 1>(row, bv0, bv1, tipL, tipR, k);
  }
}

// Lambda tiers M .. h-1: compute tier M (M > 0), then collect its bands
// ([M, M+2) and [w-M-2, w-M)) by tier parity.
template <int P, int M, int R>
__device__ __forceinline__ void fwd_collect(const double (&row)[P], double (&c0)[P], double (&c1)[P]) {
  if constexpr (R < P) {
    constexpr uint64_t m = reg_bits<P>(pair_bits(M) | pair_bits(kW - M - 2), R);
    if constexpr (m != 0) {
      if constexpr (M & 1)
        c1[R] = wave::pick(wave::lanes(m), row[R], c1[R]);
      else
        c0[R] = wave::pick(wave::lanes(m), row[R], c0[R]);
      // select here, not at the stores: deferred selects keep every tier's row live
      asm volatile("" : "+v"(c0[R]), "+v"(c1[R]));
    }
    fwd_collect<P, M, R + 1>(row, c0, c1);
  }
}

template <int P, int M>
__device__ __forceinline__ void fwd_l(double (&row)[P], double (&c0)[P], double (&c1)[P], const Consts<double>& k) {
  if constexpr (M < kH) {
    if constexpr (M > 0)
      fwd_update<P>(row, wave::dpp_move0<wave::kDppWaveShr1>(row[P - 1]), wave::dpp_move0<wave::kDppWaveShl1>(row[0]),
                    k);
    fwd_collect<P, M, 0>(row, c0, c1);
    fwd_l<P, M + 1>(row, c0, c1, k);
  }
}

// Checkpointing forward phase: the regions, tiers and slot entries that the
// reverse launch recomputes from, with P consecutive points per lane and P
// tiles per wave.  The forward keeps no history, so a lane can hold several points:
// its inner neighbours need no lane shift, and the two shifts per tier serve
// P points instead of one.  Every point gets the same update from the same
// three values, so the slots hold the same bits.
template <int P, bool HV, bool HL>
__global__ void __launch_bounds__(kW)
forward_kernel(const double* __restrict__ ustart, double* __restrict__ uT, const double* __restrict__ ck_in,
               double* __restrict__ ck_out, const Consts<double>* __restrict__ kb, int64_t n, int64_t nt, int p) {
  constexpr int LPT = kW / P;  // lanes per tile
  const int lane = threadIdx.x;
  const int l = lane % LPT;
  const int64_t j = (int64_t)blockIdx.x * P + lane / LPT;  // tile
  const bool valid = j < nt;
  const int64_t jj = valid ? j : 0;  // tiles past the end read tile 0 and store nothing
  const int64_t b = blockIdx.y;
  const Consts<double> k = kb[b];
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

  double row[P];
  if constexpr (!HV) {
#pragma unroll
    for (int r = 0; r < P; ++r) row[r] = ustart[gidx[r]];
  } else {
    // incoming band values of this lane's points, one per tier parity
    double bv0[P], bv1[P];
#pragma unroll
    for (int r = 0; r < P; ++r) {
      const int x = l * P + r;
      const int64_t src = x < kA ? sL + 2 * (x + 1) : sR + 2 * (x - kA);
      bv0[r] = ck_in[src];
      bv1[r] = ck_in[src + 1];
      row[r] = 0.0;
    }
    const double tipL = ck_in[sL + ((kH - 1) & 1)];
    const double tipR = ck_in[sR + 2 * (kW - kA) + ((kH - 1) & 1)];
    fwd_v<P, 0>(row, bv0, bv1, tipL, tipR, k);
  }
  if constexpr (HL) {
    double c0[P], c1[P];  // this lane's outgoing band values, by tier parity
#pragma unroll
    for (int r = 0; r < P; ++r) c0[r] = c1[r] = 0.0;
    fwd_l<P, 0>(row, c0, c1, k);
    if (valid) {
#pragma unroll
      for (int r = 0; r < P; ++r) {
        const int x = l * P + r;
        // left side p = x at tiers m = x-1, x; right side p = x-a+1 at m = w-x-2, w-x-1
        if (x <= kA) {
          double* const outL = ck_out + sL + 2 * x;
          if (x <= kH - 1) outL[x & 1] = (x & 1) ? c1[r] : c0[r];
          if (x >= 1) outL[(x - 1) & 1] = ((x - 1) & 1) ? c1[r] : c0[r];
        }
        if (x >= kA - 1) {
          double* const outR = ck_out + sR + 2 * (x - kA + 1);
          const int m0 = kW - x - 2, m1 = kW - x - 1;
          if (m0 >= 0) outR[m0 & 1] = (m0 & 1) ? c1[r] : c0[r];
          if (m1 <= kH - 1) outR[m1 & 1] = (m1 & 1) ? c1[r] : c0[r];
        }
      }
    }
  } else {
    if (valid) {
#pragma unroll
      for (int r = 0; r < P; ++r) uT[gidx[r]] = row[r];
    }
  }
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
  bool poison = false;        // SWEPT_DEBUG_POISON: NaN-fill checkpoints and lambda slots before use
  double* consts = nullptr;   // Consts<double>[batch]
  int Q = 1;                  // phases per checkpoint segment (1: every phase's edge state kept)
  int off = 0;                // K mod Q: the first kept phase
  int nlev = 0;               // kept checkpoint sets: phases off, off + Q, .., K - Q
  double* ckpt = nullptr;     // nlev kept sets, then Q-1 sets of the segment being recomputed;
                              // a set is batch x 2nt x 66 values
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

// Where the edge state written by phase q (the reverse launch of phase q + 1
// restarts from it) lives: the kept sets for q = off, off + Q, .., K - Q, the
// segment sets for the phases in between and below off (rewritten segment by
// segment).  The kept grid ends at K - Q so that the top segment, whose
// states the forward itself leaves in the segment sets, is a full one.
double* ckpt_set(const swept_adjoint_s* a, int q) {
  const size_t pslots = (size_t)a->batch * 2 * (size_t)a->nt * kSL;
  const int d = q - a->off;
  if (d >= 0 && d % a->Q == 0) return a->ckpt + (size_t)(d / a->Q) * pslots;
  return a->ckpt + (size_t)(a->nlev + (d % a->Q + a->Q) % a->Q - 1) * pslots;
}

// Forward phases q0 .. q1 (all with a Lambda part), each writing its own edge
// state: from the edge state of phase q0 - 1, or, for q0 = 0, from the state
// ur after the leading classic steps.
hipError_t forward_phases(const swept_adjoint_s* a, int q0, int q1, const double* ur, hipStream_t st) {
  constexpr int FP = swept::adj::kFwdPoints;
  const auto* k = reinterpret_cast<const swept::Consts<double>*>(a->consts);
  const dim3 grid((unsigned)((a->nt + FP - 1) / FP), (unsigned)a->batch);
  for (int q = q0; q <= q1; ++q) {
    if (q == 0)
      hipLaunchKernelGGL((swept::adj::forward_kernel<FP, false, true>), grid, dim3(kW), 0, st, ur, nullptr, nullptr,
                         ckpt_set(a, 0), k, a->n, a->nt, 0);
    else
      hipLaunchKernelGGL((swept::adj::forward_kernel<FP, true, true>), grid, dim3(kW), 0, st, nullptr, nullptr,
                         ckpt_set(a, q - 1), ckpt_set(a, q), k, a->n, a->nt, q);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

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
  return swept_adjoint_create_segmented(out, batch, n, dtype, dt, dx, steps, 1);
}

int swept_adjoint_create_segmented(swept_adjoint* out, int32_t batch, int64_t n, int dtype, double dt, double dx,
                                   int64_t steps, int segment) {
  if (!out) return afail(SWEPT_EINVAL, "out must not be NULL");
  *out = nullptr;
  if (batch < 1 || batch > 65535) return afail(SWEPT_EINVAL, "batch must be in [1, 65535]");
  if (dtype != SWEPT_F64) return afail(SWEPT_EUNSUPPORTED, "the adjoint is built for SWEPT_F64");
  if (n < kW || n % kW != 0) return afail(SWEPT_EUNSUPPORTED, "n must be a positive multiple of 64");
  if (steps < 1) return afail(SWEPT_EINVAL, "steps must be >= 1");
  if (!std::isfinite(dt) || !std::isfinite(dx) || dx == 0.0) return afail(SWEPT_EINVAL, "dt, dx must be finite, dx != 0");
  if (segment < 0) return afail(SWEPT_EINVAL, "segment must be >= 0");
  // the remainder steps launch one work-item per point of the batch
  const int64_t nblk = (n + swept::adj::kRemThreads - 1) / swept::adj::kRemThreads;
  if ((int64_t)batch * nblk * swept::adj::kRemThreads > (int64_t)UINT32_MAX)
    return afail(SWEPT_EUNSUPPORTED, "batch x n exceeds one launch (2^32 - 1 work-items)");
  auto* a = new (std::nothrow) swept_adjoint_s();
  if (!a) return afail(SWEPT_ENOMEM, "host allocation failed");
  a->batch = batch;
  a->n = n;
  a->steps = steps;
  a->dt = dt;
  a->dx = dx;
  a->nt = n / kW;
  a->nblk = nblk;
  a->r = (int)(steps % swept::adj::kH);
  a->K = (int)(steps / swept::adj::kH);
  // segment 0: about sqrt(K) phases per segment, which keeps about 2 sqrt(K)
  // sets instead of K for one more forward pass
  int Q = segment;
  if (Q == 0) {
    Q = 1;
    while ((int64_t)Q * Q < a->K) ++Q;
  }
  a->Q = std::max(1, std::min(Q, std::max(1, a->K)));
  a->off = a->K % a->Q;
  a->nlev = (a->K - a->off) / a->Q;
  a->poison = swept::debug_poison_requested();
  hipError_t e = hipGetDevice(&a->device);
  if (e != hipSuccess) {
    delete a;
    return ahip(e, "hipGetDevice");
  }
  const size_t state = (size_t)batch * (size_t)n * sizeof(double);
  const size_t slots = (size_t)batch * 2 * (size_t)a->nt * kSL * sizeof(double);
  a->ckpt_bytes = (size_t)(a->nlev + (a->Q > 1 ? a->Q - 1 : 0)) * slots;
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
  swept::DeviceGuard g(a->device);
  if (!g.ok) return ahip(g.err, "hipSetDevice");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int64_t total = (int64_t)a->batch * a->n;
  const size_t state = (size_t)total * sizeof(double);
  auto* k = reinterpret_cast<swept::Consts<double>*>(a->consts);
  hipLaunchKernelGGL(swept::adj::consts_kernel, dim3((unsigned)((a->batch + 63) / 64)), dim3(64), 0, st, alpha,
                     a->batch, a->dt, a->dx, k);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess && a->poison) e = swept::poison_fill(a->ckpt, a->ckpt_bytes, 8, st);
  // leading classic steps: u_0 .. u_r kept for the reverse sweep
  if (e == hipSuccess) e = hipMemcpyAsync(a->rem, u0, state, hipMemcpyDeviceToDevice, st);
  for (int m = 0; m < a->r && e == hipSuccess; ++m) {
    hipLaunchKernelGGL(swept::adj::rem_forward_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st,
                       a->rem + (size_t)m * total, a->rem + (size_t)(m + 1) * total, k, a->n, a->batch);
    e = hipGetLastError();
  }
  const double* ur = a->rem + (size_t)a->r * total;
  if (a->K == 0) {
    if (e == hipSuccess) e = hipMemcpyAsync(uT, ur, state, hipMemcpyDeviceToDevice, st);
  } else {
    for (int p = 0; p <= a->K && e == hipSuccess; ++p) {
      const double* ck_in = p > 0 ? ckpt_set(a, p - 1) : nullptr;
      double* ck_out = p < a->K ? ckpt_set(a, p) : nullptr;
      constexpr int FP = swept::adj::kFwdPoints;
      auto kern = p == 0 ? swept::adj::forward_kernel<FP, false, true>
                  : (p == a->K ? swept::adj::forward_kernel<FP, true, false> : swept::adj::forward_kernel<FP, true, true>);
      hipLaunchKernelGGL(kern, dim3((unsigned)((a->nt + FP - 1) / FP), (unsigned)a->batch), dim3(kW), 0, st, ur,
                         static_cast<double*>(uT), ck_in, ck_out, k, a->n, a->nt, p);
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
  swept::DeviceGuard g(a->device);
  if (!g.ok) return ahip(g.err, "hipSetDevice");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int64_t total = (int64_t)a->batch * a->n;
  const size_t state = (size_t)total * sizeof(double);
  auto* k = reinterpret_cast<const swept::Consts<double>*>(a->consts);
  hipError_t e = zero(a->tiles, (int64_t)a->batch * a->nt, st);
  if (e == hipSuccess) e = zero(a->rparts, (int64_t)a->batch * a->nblk, st);
  if (e == hipSuccess && a->poison)
    e = swept::poison_fill(a->lam_slots, (size_t)a->batch * 2 * (size_t)a->nt * kSL * sizeof(double), 8, st);
  // lambda at tier r: from the swept sweep (or g_uT itself when T < 32)
  double* lam_r = a->r > 0 ? a->lam_a : static_cast<double*>(g_u0);
  if (a->K == 0) {
    if (e == hipSuccess) e = hipMemcpyAsync(lam_r, g_uT, state, hipMemcpyDeviceToDevice, st);
  } else {
    const double* ur = a->rem + (size_t)a->r * total;
    for (int p = a->K; p >= 0 && e == hipSuccess; --p) {
      // entering a segment from its top (phase p kept, p - 1 not): recompute
      // the edge states of its phases from the kept state below it, or from
      // ur for the phases below the first kept one.  The top segment's
      // states are still in the segment sets from the forward.
      if (a->Q > 1 && p >= 1 && p < a->K && (p - a->off) % a->Q == 0 && p >= a->off) {
        const int q0 = p == a->off ? 0 : p - a->Q + 1;
        e = forward_phases(a, q0, p - 1, ur, st);
        if (e != hipSuccess) break;
      }
      const double* ck_in = p > 0 ? ckpt_set(a, p - 1) : nullptr;
      if (p > 0 && p < a->K) {
        constexpr int ch = swept::adj::kChain;
        hipLaunchKernelGGL(swept::adj::chain_kernel, dim3((unsigned)((a->nt + ch - 1) / ch), (unsigned)a->batch),
                           dim3(kW), 0, st, ck_in, a->lam_slots, a->tiles, k, a->nt, p, ch);
      } else {
        // the first phase (no V part) and the last (no Lambda part)
        auto kern = p == 0 ? swept::adj::region_kernel<false, true> : swept::adj::region_kernel<true, false>;
        hipLaunchKernelGGL(kern, dim3((unsigned)a->nt, (unsigned)a->batch), dim3(kW), 0, st, ur, ck_in,
                           static_cast<const double*>(g_uT), a->lam_slots, lam_r, a->tiles, k, a->n, a->nt, p);
      }
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
  swept::DeviceGuard g(a->device);
  adj_free(a);
}

}  // extern "C"
