// Per-position arithmetic of the 2D staggered elastic sweep, shared by the
// one-sweep and the multi-sweep kernels so both produce bit-identical results:
// every rounding step is spelled out (explicit fma, no compiler contraction).
#pragma once
#include <hip/hip_runtime.h>

namespace petto {
namespace el2d {

template <typename T>
__device__ __forceinline__ T fma_(T a, T b, T c) {
  return fma(a, b, c);
}

// In 2D the face forces do not depend on h: a cell's energy h^2 W(eps) with
// eps = (difference of u) / h is a quadratic form in the differences alone, so
// the sweep works with forces (stress times h) formed from displacement
// differences, and the residual sums their jumps (Eqs. 3.6, 3.9).

// Normal forces of a cell from its displacement differences d_aa = u_a(hi) - u_a(lo):
// h sigma_aa = lam (d_xx + d_yy) + 2 mu d_aa.
template <typename T>
__device__ __forceinline__ void normal_stress(T lam, T mu2, T dxx, T dyy, T& sxx, T& syy) {
  const T lt = lam * (dxx + dyy);
  sxx = fma_(mu2, dxx, lt);
  syy = fma_(mu2, dyy, lt);
}

// Engineering shear displacement of a vertex (h gamma): (ux - ux_below) + (uy - uy_left).
template <typename T>
__device__ __forceinline__ T shear_strain(T ux, T ux_below, T uy, T uy_left) {
  return (ux - ux_below) + (uy - uy_left);
}

// Shear modulus of a vertex for the divergence: mean of the four cells around it
// (absent cells carry zero), doubled on a clamped wall (the reflected ghost),
// zero when the vertex is inactive.
template <typename T>
__device__ __forceinline__ T vertex_modulus(T mu0, T e00, T e10, T e01, T e11, bool active, bool wall) {
  if (!active) return T(0);
  const T m = T(0.25) * mu0 * (((e00 + e10) + e01) + e11);
  return wall ? T(2) * m : m;
}

// Residual (force units) of a face unknown: load + normal-force jump + shear-force jump.
template <typename T>
__device__ __forceinline__ T residual(T b, T s_hi, T s_lo, T t_hi, T t_lo) {
  return (b + (s_hi - s_lo)) + (t_hi - t_lo);
}

// Damped-wave update: v <- a v + c r, u <- u + dt v.
template <typename T>
__device__ __forceinline__ void update(T ca, T cc, T dt, T r, T& u, T& v) {
  v = fma_(cc, r, ca * v);
  u = fma_(dt, v, u);
}

}  // namespace el2d
}  // namespace petto
