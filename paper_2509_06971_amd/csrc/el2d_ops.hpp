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

// Normal stresses of a cell from its strains: sigma_aa = lam tr + 2 mu eps_aa (Eq. 3.9).
template <typename T>
__device__ __forceinline__ void normal_stress(T lam, T mu2, T exx, T eyy, T& sxx, T& syy) {
  const T lt = lam * (exx + eyy);
  sxx = fma_(mu2, exx, lt);
  syy = fma_(mu2, eyy, lt);
}

// Engineering shear strain of a vertex: (ux - ux_below) / h + (uy - uy_left) / h.
template <typename T>
__device__ __forceinline__ T shear_strain(T ux, T ux_below, T uy, T uy_left, T rh) {
  return fma_(uy - uy_left, rh, (ux - ux_below) * rh);
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

// Residual (force units) of a face unknown: load + h (stress jump) + h (shear jump).
template <typename T>
__device__ __forceinline__ T residual(T b, T h, T s_hi, T s_lo, T t_hi, T t_lo) {
  return fma_(h, t_hi - t_lo, fma_(h, s_hi - s_lo, b));
}

// Damped-wave update: v <- a v + c r, u <- u + dt v.
template <typename T>
__device__ __forceinline__ void update(T ca, T cc, T dt, T r, T& u, T& v) {
  v = fma_(cc, r, ca * v);
  u = fma_(dt, v, u);
}

}  // namespace el2d
}  // namespace petto
