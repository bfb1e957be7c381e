// Device stencil arithmetic shared by every GPU kernel of the library.
//
// This is the single source of the per-point updates; the naive, LDS and
// wave-resident kernels all call these functions so that every path rounds
// identically.  Build with -ffp-contract=off and without fast-math: each
// operation below is one IEEE-754 round-to-nearest-even add, subtract or
// multiply, in the order written, or one fused multiply-add where `fmadd`
// is written (a*b + c rounded once).
//
//   heat (Sec. 4.1, Eq. HeatDisc):  Fo*(T_{i+1} + T_{i-1}) + (1-2Fo)*T_i,
//       as fmadd(Fo, T_{i+1} + T_{i-1}, (1-2Fo)*T_i)
//   KS right-hand side (Sec. 4.1, Eq. KSDisc, with the u_xx numerator read as
//   u_{i+1} + u_{i-1} - 2u_i):
//       -(((u_{i+1}^2 - u_{i-1}^2)/(4dx) + (u_{i+1} + u_{i-1} - 2u_i)/dx^2)
//         + (u_{i+2} - 4u_{i+1} + 6u_i - 4u_{i-1} + u_{i-2})/dx^4)
//     with the three divisions replaced by products with host-formed
//     inverses (Sec. 5), terms summed left to right, and each multiple of
//     u_i, u_{i+-1} inside the two difference numerators fused into the sum
//     it joins (for the multiples 2 and 4 that rounds exactly as the unfused
//     form; only 6u_i gains a rounding).  The flux difference
//     u_{i+1}^2 - u_{i-1}^2 stays unfused, so it changes sign exactly when
//     its two neighbours swap.
//   RK2 midpoint (Appendix): predictor u + (dt/2) f(u), final u + dt f(pred),
//     each one fused multiply-add.
#pragma once

#include <hip/hip_runtime.h>

namespace swept {

enum Kind : int { kHeat = 0, kKS = 1 };

// Stencil radius per tier: 3-point heat, 5-point KS (Sec. 4.3).
template <int KIND>
struct Radius {
  static constexpr int value = KIND == kHeat ? 1 : 2;
};

// Discretisation constants, formed on the host (Sec. 4.1, Sec. 5).
template <typename T>
struct Consts {
  T fo;    // heat: Fo = alpha dt / dx^2
  T c;     // heat: 1 - 2 Fo
  T i4dx;  // KS: 1/(4 dx)
  T idx2;  // KS: 1/dx^2
  T idx4;  // KS: 1/dx^4 = (1/dx^2)^2
  T dt;    // KS: dt
  T dth;   // KS: dt/2
};

// a*b + c, rounded once
__device__ __forceinline__ double fmadd(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fmadd(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

template <typename T>
__device__ __forceinline__ T heat_update(T left, T self, T right, const Consts<T>& k) {
  return fmadd(k.fo, right + left, k.c * self);
}

template <typename T>
__device__ __forceinline__ T ks_rhs(T bb, T b, T o, T a, T aa, const Consts<T>& k) {
  T nl = (a * a - b * b) * k.i4dx;
  T d2 = fmadd(T(-2), o, a + b) * k.idx2;
  T d4 = (fmadd(T(-4), b, fmadd(T(6), o, fmadd(T(-4), a, aa))) + bb) * k.idx4;
  return -((nl + d2) + d4);
}

// predictor tier: u^{m+1/2}_i from u^m at i-2..i+2
template <typename T>
__device__ __forceinline__ T ks_predictor(T bb, T b, T o, T a, T aa, const Consts<T>& k) {
  return fmadd(k.dth, ks_rhs(bb, b, o, a, aa, k), o);
}

// final tier: u^{m+1}_i from u^m_i and the predictor at i-2..i+2
template <typename T>
__device__ __forceinline__ T ks_final(T u_self, T qbb, T qb, T qo, T qa, T qaa, const Consts<T>& k) {
  return fmadd(k.dt, ks_rhs(qbb, qb, qo, qa, qaa, k), u_self);
}

}  // namespace swept
