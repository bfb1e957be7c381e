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
//   KS (Sec. 4.1, Eq. KSDisc, with the u_xx numerator read as
//   u_{i+1} + u_{i-1} - 2u_i) advanced by the RK2 midpoint rule (Appendix):
//   each stage is u - h g, with h = dt/2 (predictor, from u) or dt (final,
//   from the predictor) and
//       g = (u_{i+1} - u_{i-1})(u_{i+1} + u_{i-1})/(4dx)
//         + (u_{i+1} + u_{i-1} - 2u_i)/dx^2
//         + ((u_{i+2} + u_{i-2}) - 4(u_{i+1} + u_{i-1}) + 6u_i)/dx^4,
//   i.e. -f.  The step h is folded into the three host-formed coefficients
//   h/(4dx), h/dx^2, h/dx^4 (the divisions replaced by products, Sec. 5), and
//   with S1 = u_{i+1} + u_{i-1}, S2 = u_{i+2} + u_{i-2}:
//       h g = fmadd(h/dx^4, fmadd(6, u_i, fmadd(-4, S1, S2)),
//                   fmadd(h/dx^2, fmadd(-2, u_i, S1),
//                         (h/(4dx)) ((u_{i+1} - u_{i-1}) S1)))
//   and the stage is u - h g.  Every sum is symmetric in the two sides, the
//   flux term antisymmetric, so the update of -u(-x) is exactly the negated
//   mirror of the update of u(x).
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
  T pnl, p2, p4;  // KS predictor coefficients: (dt/2)/(4 dx), (dt/2)/dx^2, (dt/2)/dx^4
  T fnl, f2, f4;  // KS final-stage coefficients: dt/(4 dx), dt/dx^2, dt/dx^4
};

// The constants of one problem, formed in double from its dt, dx and alpha
// and rounded once to T.  Every product of two constants is formed in
// double, as h * (1/(4 dx)) and so on.
template <typename T>
inline Consts<T> make_consts(double dt, double dx, double alpha) {
  const double fo = (alpha * dt) / (dx * dx);
  const double i4dx = 1.0 / (4.0 * dx), idx2 = 1.0 / (dx * dx), idx4 = idx2 * idx2;
  const double dth = 0.5 * dt;
  Consts<T> k;
  k.fo = (T)fo;
  k.c = (T)(1.0 - 2.0 * fo);
  k.i4dx = (T)i4dx;
  k.idx2 = (T)idx2;
  k.idx4 = (T)idx4;
  k.dt = (T)dt;
  k.dth = (T)dth;
  k.pnl = (T)(dth * i4dx);
  k.p2 = (T)(dth * idx2);
  k.p4 = (T)(dth * idx4);
  k.fnl = (T)(dt * i4dx);
  k.f2 = (T)(dt * idx2);
  k.f4 = (T)(dt * idx4);
  return k;
}

// a*b + c, rounded once
__device__ __forceinline__ double fmadd(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fmadd(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

template <typename T>
__device__ __forceinline__ T heat_update(T left, T self, T right, const Consts<T>& k) {
  return fmadd(k.fo, right + left, k.c * self);
}

// h g at one point from u at i-2 .. i+2 (see the header), given the
// stage's coefficients cnl = h/(4dx), c2 = h/dx^2, c4 = h/dx^4.
template <typename T>
__device__ __forceinline__ T ks_hg(T bb, T b, T o, T a, T aa, T cnl, T c2, T c4) {
  const T s1 = a + b, s2 = aa + bb;
  const T flux = (a - b) * s1;
  const T d2 = fmadd(T(-2), o, s1);
  const T d4 = fmadd(T(6), o, fmadd(T(-4), s1, s2));
  return fmadd(c4, d4, fmadd(c2, d2, cnl * flux));
}

// predictor tier: u^{m+1/2}_i from u^m at i-2..i+2
template <typename T>
__device__ __forceinline__ T ks_predictor(T bb, T b, T o, T a, T aa, const Consts<T>& k) {
  return o - ks_hg(bb, b, o, a, aa, k.pnl, k.p2, k.p4);
}

// final tier: u^{m+1}_i from u^m_i and the predictor at i-2..i+2
template <typename T>
__device__ __forceinline__ T ks_final(T u_self, T qbb, T qb, T qo, T qa, T qaa, const Consts<T>& k) {
  return u_self - ks_hg(qbb, qb, qo, qa, qaa, k.fnl, k.f2, k.f4);
}

}  // namespace swept
