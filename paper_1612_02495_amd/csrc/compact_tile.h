// One swept phase of one 64-lane tile with the active region compacted onto
// fewer points per lane (the compacted wave engine).
//
// The swept rule's V part grows from nothing to the full tile and its
// Lambda part shrinks back (Sec. 4.2), so a wave that always spans the whole
// tile leaves about half of its lanes on don't-care points.  Here the part of
// the tile that a run of tiers touches is laid out over all 64 lanes with R
// contiguous points per lane, R = 4, 8, .., P (see Step below).  A layout R
// covers the 64 R points centred on the tile middle,
// x in [32 (P - R), 32 (P + R)).  The V part starts in the narrowest layout
// and widens as its gap grows, the Lambda part starts in the full layout and
// narrows as its triangle climbs; each change of layout passes the live row
// through LDS.  Within one layout the tier code is the register engine's
// (wave_tile.h) on a 64-lane tile with its seam at lane 32.
//
// The edge bands live in LDS for the whole phase, position-major
// sb[(x + S) * 2 + (tier & 1)] for x in [-S, 64 P + S): the incoming slots
// are copied in before the V part and the outgoing slots copied out after the
// Lambda part, so the slot contents are exactly those of the register engine
// and both engines can run alternate phases of one run.  Each layout loads
// the band values of its own points into registers (V) or merges the values
// its tiers collect back into LDS (Lambda).
#pragma once

#include "wave_tile.h"

namespace swept {
namespace compact {

// Ordering of LDS accesses inside one tile.  A tile belongs to one wave and
// so do its LDS buffers; the LDS operations of one wave execute in order, so
// a wavefront-scope fence, which keeps the compiler from moving LDS accesses
// across it, is all a layout change needs.  (In the batched kernel several
// waves of a workgroup change layout at different times, so a workgroup
// barrier there could even pair up different layout changes.)
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// LDS index with one spare value every 32, which spreads lane-strided
// accesses over more banks.
__host__ __device__ constexpr int pad(int i) { return i + (i >> 5); }

// Layouts grow in steps of 4 points per lane for both stencils.  (The
// 5-point stencil needs a multiple of 4 so that every layout holds whole KS
// step pairs.  For heat, steps of 2 leave fewer idle lanes but pay twice the
// layout changes and twice the unrolled code; on MI355X the heat FP64 N=2^20
// diamond ran at 4.40e12 cell-updates/s with steps of 2, 4.44e12 with 4 and
// 4.12e12 with 8, FP32 5.40e12 / 5.74e12 / 5.16e12.)
template <int KIND>
struct Step {
  static constexpr int value = 4;
};

// LDS values of the band buffer and of the relayout staging row.
template <int KIND, int P>
struct Lds {
  static constexpr int S = Radius<KIND>::value;
  static constexpr int band = pad(2 * (64 * P + 2 * S) - 1) + 1;
  static constexpr int stage = pad(64 * P - 1) + 1;
};

// V tiers of block b in a layout of R points per lane whose seam is at lane
// 32: all B tiers (FULL) or those below t1.  Left band of tier t:
// [-S(t+2), -S t) from the seam, lanes 31-b and 30-b; right band
// [S t, S(t+2)), lanes 32+b and 33+b.
template <int KIND, typename T, int R, bool FULL, bool TIPS, bool INS = false>
__device__ __forceinline__ void v_blk(T (&A)[R], T (&Q)[R], const T (&buf)[R][2], int b, int t1, int lane,
                                      const T (&tipL)[Radius<KIND>::value],
                                      const T (&tipR)[Radius<KIND>::value], const Consts<T>& k,
                                      wave::Ends e = wave::Ends{}) {
  constexpr int S = Radius<KIND>::value;
  constexpr int B = R / S;
  const bool mL0 = lane == 31 - b, mL1 = lane == 30 - b;
  const bool mR0 = lane == 32 + b, mR1 = lane == 33 + b;
  const bool first = lane == 0, last = lane == 63;
#pragma unroll
  for (int j = 0; j < B; ++j) {
    const int t = b * B + j;
    if (FULL || t < t1) {
      T(&row)[R] = KIND == kHeat ? A : wave::row_of<T, R>(A, Q, j & 1);
#pragma unroll
      for (int i = 0; i < 2 * S; ++i) {
        const int ol = R - S * (j + 2) + i;  // offset from lane 31-b
        const int rl = (ol + R) % R;
        row[rl] = wave::pick(ol < 0 ? mL1 : mL0, buf[rl][j & 1], row[rl]);
        const int orr = S * j + i;  // offset from lane 32+b
        const int rr = orr % R;
        row[rr] = wave::pick(orr >= R ? mR1 : mR0, buf[rr][j & 1], row[rr]);
      }
      wave::tier<KIND, T, R, TIPS, INS>(A, Q, ((j + 1) & 1) != 0, tipL, tipR, first, last, k, e);
    }
  }
}

// V tiers [t0, t1) with t0 a multiple of the block height: whole blocks, then
// the guarded remainder (with the triangle tips when TIPS).
template <int KIND, typename T, int R, bool TIPS, bool INS = false>
__device__ __forceinline__ void v_run(T (&A)[R], T (&Q)[R], const T (&buf)[R][2], int t0, int t1, int lane,
                                      const T (&tipL)[Radius<KIND>::value],
                                      const T (&tipR)[Radius<KIND>::value], const Consts<T>& k,
                                      wave::Ends e = wave::Ends{}) {
  constexpr int B = R / Radius<KIND>::value;
  if (t0 >= t1) return;
  const int bl = (t1 - 1) / B;  // block holding the last tier
  for (int b = t0 / B; b < bl; ++b) v_blk<KIND, T, R, true, false, INS>(A, Q, buf, b, t1, lane, tipL, tipR, k, e);
  v_blk<KIND, T, R, false, TIPS, INS>(A, Q, buf, bl, t1, lane, tipL, tipR, k, e);
}

// Lambda tiers of block b, counted from the base of the layout's own 64 R-
// point tile: all B tiers (FULL) or those in [t0, t1).  Each collects the band
// values of tier t ([S t, S t + 2S), lanes b and b+1; [64 R - S(t+2),
// 64 R - S t), lanes 63-b and 62-b), then computes tier t+1 unless
// t == tskip (the empty top of a full triangle; never inside a FULL block).
// SEL: collect the left band only where colL and the right band only where
// colR (a tile of uneven width collects its two bands in two passes).
template <int KIND, typename T, int R, bool FULL, bool INS = false, bool SEL = false>
__device__ __forceinline__ void l_blk(T (&A)[R], T (&Q)[R], T (&buf)[R][2], int b, int t0, int t1, int tskip,
                                      int lane, const Consts<T>& k, wave::Ends e = wave::Ends{}, bool colL = true,
                                      bool colR = true) {
  constexpr int S = Radius<KIND>::value;
  constexpr int B = R / S;
  const bool cl = !SEL || colL, cr = !SEL || colR;
  const bool mL0 = cl && lane == b, mL1 = cl && lane == b + 1;
  const bool mR0 = cr && lane == 63 - b, mR1 = cr && lane == 62 - b;
  const T tip0[S] = {};
#pragma unroll
  for (int j = 0; j < B; ++j) {
    const int t = b * B + j;
    if (FULL || (t >= t0 && t < t1)) {
      T(&row)[R] = KIND == kHeat ? A : wave::row_of<T, R>(A, Q, j & 1);
#pragma unroll
      for (int i = 0; i < 2 * S; ++i) {
        const int ol = S * j + i;  // offset from lane b
        const int rl = ol % R;
        buf[rl][j & 1] = wave::pick(ol >= R ? mL1 : mL0, row[rl], buf[rl][j & 1]);
        const int orr = R - S * (j + 2) + i;  // offset from lane 63-b
        const int rr = (orr + R) % R;
        buf[rr][j & 1] = wave::pick(orr < 0 ? mR1 : mR0, row[rr], buf[rr][j & 1]);
      }
      if (FULL || t != tskip)
        wave::tier<KIND, T, R, false, INS>(A, Q, ((j + 1) & 1) != 0, tip0, tip0, false, false, k, e);
    }
  }
}

// Lambda tiers [t0, t1) of a layout: a guarded head block when t0 is not a
// block boundary, whole blocks, then the guarded remainder.
template <int KIND, typename T, int R, bool INS = false, bool SEL = false>
__device__ __forceinline__ void l_run(T (&A)[R], T (&Q)[R], T (&buf)[R][2], int t0, int t1, int tskip, int lane,
                                      const Consts<T>& k, wave::Ends e = wave::Ends{}, bool colL = true,
                                      bool colR = true) {
  constexpr int B = R / Radius<KIND>::value;
  if (t1 <= t0) return;
  int b = t0 / B;
  const int bl = (t1 - 1) / B;
  if (t0 % B != 0 && b < bl) {
    l_blk<KIND, T, R, false, INS, SEL>(A, Q, buf, b, t0, t1, tskip, lane, k, e, colL, colR);
    ++b;
  }
  for (; b < bl; ++b) l_blk<KIND, T, R, true, INS, SEL>(A, Q, buf, b, t0, t1, -1, lane, k, e, colL, colR);
  l_blk<KIND, T, R, false, INS, SEL>(A, Q, buf, bl, t0, t1, tskip, lane, k, e, colL, colR);
}

// Where a tile of an insulated rod holds the rod's ends (all false for the
// tiles in between): `seam` -- the ends meet at the tile middle (the shifted
// tiling's tile across the ring seam: node n-1 is point 32P-1, node 0 is
// point 32P); `lo` -- node 0 is the tile's first point; `hi` -- node n-1 is
// its last point.
struct Bnd {
  bool seam = false;
  bool lo = false;
  bool hi = false;
};

// Lanes of layout R (window centred on the tile middle) holding an end: the
// middle is lane 31's last and lane 32's first point in every layout; the
// tile's first and last points are in the full layout only.
template <int P, int R>
__device__ __forceinline__ wave::Ends ends_of(const Bnd& bd, int lane) {
  wave::Ends e;
  e.left = (bd.seam && lane == 32) || (R == P && bd.lo && lane == 0);
  e.right = (bd.seam && lane == 31) || (R == P && bd.hi && lane == 63);
  return e;
}

// V layouts R, R + step, .., P - step.  `done` counts the V tiers already
// computed; the row travels between layouts through stg.
template <int KIND, typename T, int P, int R, bool INS = false>
__device__ __forceinline__ void v_narrow(T* sb, T* stg, int hv, int& done, int lane, const Consts<T>& k,
                                         const Bnd& bd = Bnd{}) {
  if constexpr (R < P) {
    constexpr int S = Radius<KIND>::value;
    // The layout holds the tiers whose band fits, S (t + 2) <= 32 R; it hands
    // over on a block boundary of the next layout (for KS an even tier).
    constexpr int BN = (R + Step<KIND>::value) / S;
    constexpr int kEnd = (32 * R / S - 1) / BN * BN;
    const int tend = hv < kEnd ? hv : kEnd;
    if (done < tend) {
      const int xl = 32 * (P - R) + lane * R;
      T A[R], Q[R], buf[R][2];
#pragma unroll
      for (int r = 0; r < R; ++r) {
        A[r] = done > 0 ? stg[pad(xl + r)] : T(0);
        Q[r] = T(0);
        buf[r][0] = sb[pad(2 * (xl + r + S))];
        buf[r][1] = sb[pad(2 * (xl + r + S) + 1)];
      }
      const T tip0[S] = {};
      v_run<KIND, T, R, false, INS>(A, Q, buf, done, tend, lane, tip0, tip0, k, ends_of<P, R>(bd, lane));
      done = tend;
      wave_sync();  // every lane has read its row before the row is rewritten
#pragma unroll
      for (int r = 0; r < R; ++r) stg[pad(xl + r)] = A[r];
      wave_sync();
    }
    v_narrow<KIND, T, P, R + Step<KIND>::value, INS>(sb, stg, hv, done, lane, k, bd);
  }
}

// Lambda layouts R, R - step, .., step, entered at tier `done` (a multiple of
// 32 step / S, where the triangle first fits the next narrower layout).
template <int KIND, typename T, int P, int R, bool INS = false>
__device__ __forceinline__ void l_narrow(T* sb, T* stg, int hl, bool empty_top, int& done, int lane,
                                         const Consts<T>& k, const Bnd& bd = Bnd{}) {
  if constexpr (R > 0) {
    constexpr int S = Radius<KIND>::value;
    constexpr int ST = Step<KIND>::value;
    constexpr int kFirst = 32 * (P - R) / S;  // first tier of this layout
    constexpr int kNext = R > ST ? 32 * (P - R + ST) / S : 1 << 30;
    if (done < hl) {
      const int tend = hl < kNext ? hl : kNext;
      const int xl = 32 * (P - R) + lane * R;
      T A[R], Q[R], buf[R][2];
#pragma unroll
      for (int r = 0; r < R; ++r) {
        A[r] = stg[pad(xl + r)];
        Q[r] = T(0);
        buf[r][0] = sb[pad(2 * (xl + r + S))];
        buf[r][1] = sb[pad(2 * (xl + r + S) + 1)];
      }
      // entered at its first tier (done == kFirst): virtual tiers from 0
      const int tskip = empty_top ? hl - 1 - kFirst : -1;
      l_run<KIND, T, R, INS>(A, Q, buf, 0, tend - kFirst, tskip, lane, k, ends_of<P, R>(bd, lane));
      done = tend;
      if (done >= hl && !empty_top) {
        // flat top of the trapezoid: the row at its top tier
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const int x = xl + r;
          if (x >= S * hl && x < 64 * P - S * hl) {
            if (hl & 1)
              buf[r][1] = A[r];
            else
              buf[r][0] = A[r];
          }
        }
      }
      wave_sync();  // all reads of this layout's rows precede the writes
#pragma unroll
      for (int r = 0; r < R; ++r) {
        sb[pad(2 * (xl + r + S))] = buf[r][0];
        sb[pad(2 * (xl + r + S) + 1)] = buf[r][1];
        if (done < hl) stg[pad(xl + r)] = A[r];
      }
      wave_sync();
    }
    l_narrow<KIND, T, P, R - ST, INS>(sb, stg, hl, empty_top, done, lane, k, bd);
  }
}

// ROLE: 0 up-triangle (hv == 0), 1 diamond, 2 down-triangle (hl == 0).  The
// tile is 64 P points from `origin`, seam at 32 P; sL/sR are its left and
// right edge slots (layout as in wave_tile.h with kL = kR = 32).  INS: heat on
// an insulated rod, with the rod's ends in this tile where `bd` says.
template <int KIND, typename T, int P, int ROLE, bool INS = false>
__device__ __forceinline__ void tile_phase(T* u, int64_t n, int64_t origin, T* sL, T* sR, int hv, int hl,
                                           const Consts<T>& k, int lane, T* sb, T* stg, const Bnd& bd = Bnd{}) {
  constexpr int S = Radius<KIND>::value;
  constexpr int W = 64 * P;
  constexpr int HALF = 32 * P;
  constexpr int ST = Step<KIND>::value;
  constexpr int SV = 2 * (HALF + S);  // values of one slot that a phase reads or writes

  T A[P];
  T Q[P];
  T buf[P][2];
#pragma unroll
  for (int r = 0; r < P; ++r) Q[r] = T(0);

  if constexpr (ROLE == 0) {
#pragma unroll
    for (int r = 0; r < P; ++r) {
      int64_t g2 = origin + lane * P + r;
      if (g2 >= n) g2 -= n;
      A[r] = u[g2];
    }
  } else {
    // incoming slots: consumer left input p = x + S, right input p = x - HALF;
    // every load is issued before the first LDS store
    {
      constexpr int NIT = (SV + 63) / 64;
      T inL[NIT], inR[NIT];
#pragma unroll
      for (int it = 0; it < NIT; ++it) {
        const int i = it * 64 + lane;
        inL[it] = i < SV ? sL[i] : T(0);
        inR[it] = i < SV ? sR[i] : T(0);
      }
#pragma unroll
      for (int it = 0; it < NIT; ++it) {
        const int i = it * 64 + lane;
        if (i < SV) {
          sb[pad(i)] = inL[it];
          sb[pad(SV + i)] = inR[it];
        }
      }
    }
    wave_sync();
    int done = 0;
    v_narrow<KIND, T, P, ST, INS>(sb, stg, hv, done, lane, k, bd);
#pragma unroll
    for (int r = 0; r < P; ++r) {
      A[r] = done > 0 ? stg[pad(lane * P + r)] : T(0);
      buf[r][0] = sb[pad(2 * (lane * P + r + S))];
      buf[r][1] = sb[pad(2 * (lane * P + r + S) + 1)];
    }
    // triangle tips beyond the tile ends, used by the last tier of a full V
    T tipL[S], tipR[S];
    const int tp = (hv - 1) & 1;
#pragma unroll
    for (int i = 0; i < S; ++i) {
      tipL[i] = sb[pad(2 * i + tp)];
      tipR[i] = sb[pad(2 * (W + S + i) + tp)];
    }
    v_run<KIND, T, P, true, INS>(A, Q, buf, done, hv, lane, tipL, tipR, k, ends_of<P, P>(bd, lane));
    // flat tops of the producer trapezoids: tile points outside the gap
    if (S * hv < HALF) {
#pragma unroll
      for (int r = 0; r < P; ++r) {
        const int x = lane * P + r;
        if (x < HALF - S * hv || x >= HALF + S * hv) A[r] = wave::pick((hv & 1) != 0, buf[r][1], buf[r][0]);
      }
    }
    wave_sync();  // the V's reads of sb and stg precede the Lambda's writes
  }

  if constexpr (ROLE == 2) {
#pragma unroll
    for (int r = 0; r < P; ++r) {
      int64_t g2 = origin + lane * P + r;
      if (g2 >= n) g2 -= n;
      u[g2] = A[r];
    }
  } else {
#pragma unroll
    for (int r = 0; r < P; ++r) {
      buf[r][0] = T(0);
      buf[r][1] = T(0);
    }
    const bool empty_top = 2 * S * hl >= W;
    constexpr int kNext = P > ST ? 32 * ST / S : 1 << 30;
    const int tend = hl < kNext ? hl : kNext;
    const int tskip = empty_top ? hl - 1 : -1;
    l_run<KIND, T, P, INS>(A, Q, buf, 0, tend, tskip, lane, k, ends_of<P, P>(bd, lane));
    int done = tend;
    if (done >= hl && !empty_top) {
#pragma unroll
      for (int r = 0; r < P; ++r) {
        const int x = lane * P + r;
        if (x >= S * hl && x < W - S * hl) {
          if (hl & 1)
            buf[r][1] = A[r];
          else
            buf[r][0] = A[r];
        }
      }
    }
#pragma unroll
    for (int r = 0; r < P; ++r) {
      sb[pad(2 * (lane * P + r + S))] = buf[r][0];
      sb[pad(2 * (lane * P + r + S) + 1)] = buf[r][1];
      if (done < hl) stg[pad(lane * P + r)] = A[r];
    }
    wave_sync();
    l_narrow<KIND, T, P, P - ST, INS>(sb, stg, hl, empty_top, done, lane, k, bd);
    // outgoing slots: producer left side p = x (x < HALF + S), right side
    // p = x - HALF + S (x >= HALF - S)
    {
      constexpr int NIT = (SV + 63) / 64;
      T outL[NIT], outR[NIT];
#pragma unroll
      for (int it = 0; it < NIT; ++it) {
        const int i = it * 64 + lane;
        outL[it] = i < SV ? sb[pad(2 * S + i)] : T(0);
        outR[it] = i < SV ? sb[pad(2 * HALF + i)] : T(0);
      }
#pragma unroll
      for (int it = 0; it < NIT; ++it) {
        const int i = it * 64 + lane;
        if (i < SV) {
          sL[i] = outL[it];
          sR[i] = outR[it];
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Tiles with uneven halves (the batched kernel, and single grids whose size no
// tile width divides): wL and wR points left and right of the seam (1 .. 32 P
// each), w = wL + wR, seam a = wL.  The V layouts are centred on the seam as
// above, so their band positions are compile-time for any a.  The Lambda
// triangle of tier t is [S t, w - S t).  Layout R is entered at the even tier
// f = the smallest even tier at which the triangle fits 64 R points, with its
// window [S f, S f + 64 R) at the triangle's left end, so its virtual tiers
// t - f have the parity of the true tiers (the slot parity, and for KS the
// predictor/final alternation, follow it) and its left band sits at
// compile-time positions.  Its right band does too when the window is exactly
// as wide as the triangle at tier f, which holds when w is a multiple of 4S.
// Otherwise the triangle is climbed twice from the same base row: once in
// these windows collecting the left band, once in windows ending at the
// triangle's right end, [w - S f - 64 R, w - S f), collecting the right band;
// each pass merges only its own side of the tile (x < w/2, x >= w/2) into the
// band buffer.  Between the passes the base row waits in the tile's own span
// of u, which no tile reads or writes between the up and the down phase.
// Layout points outside the tile are don't-care: their LDS loads read zero
// and their stores are skipped.

// Tiling of a ring of n points into 2 nt halves for tiles of at most 64 P
// points: every half but the last is `base` or `base + q` points with
// q = 4 S (a multiple of q), the last half takes the rest (`last`, base ..
// base + q - 1 points), so every tile but the two holding the last half has a
// width that is a multiple of 4 S.  nt = ceil(n / (64 P - 2 q)) keeps every
// half within 32 P points.
struct Uneven {
  int64_t nt;
  int64_t base;   // width of the narrowest halves (a multiple of q)
  int64_t extra;  // halves 0 .. extra-1 are base + q wide
  int64_t last;   // width of half 2 nt - 1
  int q;
};

__host__ __device__ constexpr int64_t ceil_div64(int64_t x, int64_t d) {
  return x >= 0 ? (x + d - 1) / d : -((-x) / d);
}

__host__ __device__ inline Uneven uneven_tiling(int64_t n, int P, int S) {
  Uneven t{};
  t.q = 4 * S;
  t.nt = ceil_div64(n, 64 * P - 2 * t.q);
  const int64_t h = n / (2 * t.nt);
  t.base = t.q * (h / t.q);
  const int64_t r = n - 2 * t.nt * t.base;
  t.extra = r / t.q;
  t.last = t.base + r % t.q;
  return t;
}

// First point (from the ring's point 0) and width of half i.
__host__ __device__ inline int64_t uneven_origin(const Uneven& t, int64_t i) {
  return i * t.base + t.q * (i < t.extra ? i : t.extra);
}
__host__ __device__ inline int uneven_width(const Uneven& t, int64_t i) {
  return (int)(i == 2 * t.nt - 1 ? t.last : t.base + (i < t.extra ? t.q : 0));
}

// Tiers of a full phase of the tiling: the narrowest half's triangle (whole
// KS steps).
__host__ __device__ inline int uneven_full_tiers(const Uneven& t, int S) {
  int h = (int)(t.base / S);
  if (S == 2) h &= ~1;
  return h;
}

struct GTile {
  int w;  // tile points
  int a;  // seam
};

__device__ __forceinline__ bool in_tile(int x, int w) { return (unsigned)x < (unsigned)w; }

// The even tier where Lambda layout R of a w-point tile starts (see above).
template <int KIND>
__device__ __forceinline__ int l_entry(int w, int R) {
  const int f = (int)ceil_div64(w - 64 * R, 2 * Radius<KIND>::value);
  return f + (f & 1);
}

template <int KIND, typename T>
__device__ __forceinline__ T band_ld(const T* sb, int x, int q, int w) {
  constexpr int S = Radius<KIND>::value;
  return (x >= -S && x < w + S) ? sb[pad(2 * (x + S) + q)] : T(0);
}

template <int KIND, typename T, int P, int R>
__device__ __forceinline__ void v_narrow_g(T* sb, T* stg, const GTile& g, int hv, int& done, int lane,
                                           const Consts<T>& k) {
  if constexpr (R < P) {
    constexpr int S = Radius<KIND>::value;
    constexpr int BN = (R + Step<KIND>::value) / S;
    constexpr int kEnd = (32 * R / S - 1) / BN * BN;
    const int tend = hv < kEnd ? hv : kEnd;
    if (done < tend) {
      const int xl = g.a - 32 * R + lane * R;
      T A[R], Q[R], buf[R][2];
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int x = xl + r;
        A[r] = (done > 0 && in_tile(x, g.w)) ? stg[pad(x)] : T(0);
        Q[r] = T(0);
        buf[r][0] = band_ld<KIND>(sb, x, 0, g.w);
        buf[r][1] = band_ld<KIND>(sb, x, 1, g.w);
      }
      const T tip0[S] = {};
      v_run<KIND, T, R, false>(A, Q, buf, done, tend, lane, tip0, tip0, k);
      done = tend;
      wave_sync();
#pragma unroll
      for (int r = 0; r < R; ++r)
        if (in_tile(xl + r, g.w)) stg[pad(xl + r)] = A[r];
      wave_sync();
    }
    v_narrow_g<KIND, T, P, R + Step<KIND>::value>(sb, stg, g, hv, done, lane, k);
  }
}

// Lambda layouts R, R - step, .., step (those not wider than the first one,
// r0); the row arrives in stg.  `done` counts the Lambda tiers computed.
// mode 0: both bands, windows at the triangle's left end; 1: the left band
// only, same windows; 2: the right band only, windows at the right end.
// Only points in [lo, hi) are merged into the band buffer.
template <int KIND, typename T, int P, int R>
__device__ __forceinline__ void l_narrow_g(T* sb, T* stg, const GTile& g, int r0, int hl, bool empty_top, int& done,
                                           int lane, const Consts<T>& k, int mode, int lo, int hi) {
  if constexpr (R > 0) {
    constexpr int S = Radius<KIND>::value;
    constexpr int ST = Step<KIND>::value;
    if (R <= r0 && done < hl) {
      const int first = l_entry<KIND>(g.w, R);  // tier where this layout's window starts
      const int next = R > ST ? l_entry<KIND>(g.w, R - ST) : (1 << 30);
      const int tend = hl < next ? hl : next;
      const int base = mode == 2 ? g.w - S * first - 64 * R : S * first;
      const int xl = base + lane * R;
      T A[R], Q[R], buf[R][2];
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int x = xl + r;
        A[r] = in_tile(x, g.w) ? stg[pad(x)] : T(0);
        Q[r] = T(0);
        buf[r][0] = R == r0 ? T(0) : band_ld<KIND>(sb, x, 0, g.w);
        buf[r][1] = R == r0 ? T(0) : band_ld<KIND>(sb, x, 1, g.w);
      }
      const int tskip = empty_top ? hl - 1 - first : -1;
      l_run<KIND, T, R, false, true>(A, Q, buf, done - first, tend - first, tskip, lane, k, wave::Ends{}, mode != 2,
                                     mode != 1);
      done = tend;
      if (done >= hl && !empty_top) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const int x = xl + r;
          if (x >= S * hl && x < g.w - S * hl) {
            if (hl & 1)
              buf[r][1] = A[r];
            else
              buf[r][0] = A[r];
          }
        }
      }
      wave_sync();
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int x = xl + r;
        if (in_tile(x, g.w)) {
          if (x >= lo && x < hi) {
            sb[pad(2 * (x + S))] = buf[r][0];
            sb[pad(2 * (x + S) + 1)] = buf[r][1];
          }
          if (done < hl) stg[pad(x)] = A[r];
        }
      }
      wave_sync();
    }
    l_narrow_g<KIND, T, P, R - ST>(sb, stg, g, r0, hl, empty_top, done, lane, k, mode, lo, hi);
  }
}

// One phase of one uneven tile: hv V tiers (0: read the row from u), then hl
// Lambda tiers (0: write the row to u).  The tile is wL + wR points from
// `origin` (ring index, wrapped mod n), seam at wL; sL/sR are its edge slots
// (layout as in wave_tile.h, positions in points); sb and stg this wave's LDS
// band buffer and staging row.  hv and hl must not exceed min(wL, wR) / S.
template <int KIND, typename T, int P>
__device__ __forceinline__ void tile_phase_g(T* u, int64_t n, int64_t origin, T* sL, T* sR, int wL, int wR, int hv,
                                             int hl, const Consts<T>& k, int lane, T* sb, T* stg) {
  constexpr int S = Radius<KIND>::value;
  constexpr int ST = Step<KIND>::value;
  constexpr int NV = (2 * (32 * P + S) + 63) / 64;  // copy iterations per slot side
  GTile g;
  g.w = wL + wR;
  g.a = wL;
  const int nL = 2 * (g.a + S), nR = 2 * (g.w - g.a + S);  // slot values read or written per side

  if (hv == 0) {
    T in[P];
#pragma unroll
    for (int it = 0; it < P; ++it) {
      const int x = it * 64 + lane;
      int64_t g2 = origin + x;
      if (g2 >= n) g2 -= n;
      in[it] = x < g.w ? u[g2] : T(0);
    }
#pragma unroll
    for (int it = 0; it < P; ++it) {
      const int x = it * 64 + lane;
      if (x < g.w) stg[pad(x)] = in[it];
    }
    wave_sync();
  } else {
    {
      T inL[NV], inR[NV];
#pragma unroll
      for (int it = 0; it < NV; ++it) {
        const int i = it * 64 + lane;
        inL[it] = i < nL ? sL[i] : T(0);
        inR[it] = i < nR ? sR[i] : T(0);
      }
#pragma unroll
      for (int it = 0; it < NV; ++it) {
        const int i = it * 64 + lane;
        if (i < nL) sb[pad(i)] = inL[it];
        if (i < nR) sb[pad(nL + i)] = inR[it];
      }
    }
    wave_sync();
    int done = 0;
    v_narrow_g<KIND, T, P, ST>(sb, stg, g, hv, done, lane, k);
    const int xl = g.a - 32 * P + lane * P;
    T A[P], Q[P], buf[P][2];
#pragma unroll
    for (int r = 0; r < P; ++r) {
      const int x = xl + r;
      A[r] = (done > 0 && in_tile(x, g.w)) ? stg[pad(x)] : T(0);
      Q[r] = T(0);
      buf[r][0] = band_ld<KIND>(sb, x, 0, g.w);
      buf[r][1] = band_ld<KIND>(sb, x, 1, g.w);
    }
    T tipL[S], tipR[S];
    const int tp = (hv - 1) & 1;
#pragma unroll
    for (int i = 0; i < S; ++i) {
      tipL[i] = sb[pad(2 * i + tp)];
      tipR[i] = sb[pad(2 * (g.w + S + i) + tp)];
    }
    v_run<KIND, T, P, true>(A, Q, buf, done, hv, lane, tipL, tipR, k);
    // flat tops of the producer trapezoids: tile points outside the gap
#pragma unroll
    for (int r = 0; r < P; ++r) {
      const int x = xl + r;
      if (x < g.a - S * hv || x >= g.a + S * hv) A[r] = wave::pick((hv & 1) != 0, buf[r][1], buf[r][0]);
    }
    wave_sync();  // the V's reads of sb and stg precede the writes below
    if (hl == 0) {
#pragma unroll
      for (int r = 0; r < P; ++r) {
        const int x = xl + r;
        if (in_tile(x, g.w)) {
          int64_t g2 = origin + x;
          if (g2 >= n) g2 -= n;
          u[g2] = A[r];
        }
      }
      return;
    }
#pragma unroll
    for (int r = 0; r < P; ++r)
      if (in_tile(xl + r, g.w)) stg[pad(xl + r)] = A[r];
    wave_sync();
  }
  // narrowest layout whose window holds the whole base: 64 r0 >= w
  const int r0 = (int)ceil_div64(g.w, 64 * ST) * ST;
  const bool empty_top = 2 * S * hl >= g.w;
  if (g.w % (4 * S) == 0) {
    int done = 0;
    l_narrow_g<KIND, T, P, P>(sb, stg, g, r0, hl, empty_top, done, lane, k, 0, 0, g.w);
  } else {
    // two passes from the same base row, parked in the tile's span of u
    const int split = g.w / 2;
#pragma unroll
    for (int it = 0; it < P; ++it) {
      const int x = it * 64 + lane;
      if (x < g.w) {
        int64_t g2 = origin + x;
        if (g2 >= n) g2 -= n;
        u[g2] = stg[pad(x)];
      }
    }
    int done = 0;
    l_narrow_g<KIND, T, P, P>(sb, stg, g, r0, hl, empty_top, done, lane, k, 1, 0, split);
    T row[P];
#pragma unroll
    for (int it = 0; it < P; ++it) {
      const int x = it * 64 + lane;
      int64_t g2 = origin + x;
      if (g2 >= n) g2 -= n;
      row[it] = x < g.w ? u[g2] : T(0);
    }
#pragma unroll
    for (int it = 0; it < P; ++it) {
      const int x = it * 64 + lane;
      if (x < g.w) stg[pad(x)] = row[it];
    }
    wave_sync();
    done = 0;
    l_narrow_g<KIND, T, P, P>(sb, stg, g, r0, hl, empty_top, done, lane, k, 2, split, g.w);
  }
  // outgoing slots: producer left side p = x (x < a + S), right side
  // p = x - a + S (x >= a - S)
  {
    T oL[NV], oR[NV];
#pragma unroll
    for (int it = 0; it < NV; ++it) {
      const int i = it * 64 + lane;
      oL[it] = i < nL ? sb[pad(2 * S + i)] : T(0);
      oR[it] = i < nR ? sb[pad(2 * g.a + i)] : T(0);
    }
#pragma unroll
    for (int it = 0; it < NV; ++it) {
      const int i = it * 64 + lane;
      if (i < nL) sL[i] = oL[it];
      if (i < nR) sR[i] = oR[it];
    }
  }
}

}  // namespace compact
}  // namespace swept
