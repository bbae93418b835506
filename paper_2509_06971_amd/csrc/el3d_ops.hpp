// Per-unknown arithmetic of the 3D staggered elastic sweep, with every rounding
// step spelled out (explicit fma, no compiler contraction).
#pragma once
#include <hip/hip_runtime.h>

namespace petto {
namespace el3d {

// Normal stresses of a cell: sigma_aa = lam tr + 2 mu eps_aa (Eq. 3.9 in 3D).
template <typename T>
__device__ __forceinline__ void normal_stress(T lam, T mu2, T exx, T eyy, T ezz, T& sxx, T& syy, T& szz) {
  const T lt = lam * ((exx + eyy) + ezz);
  sxx = fma(mu2, exx, lt);
  syy = fma(mu2, eyy, lt);
  szz = fma(mu2, ezz, lt);
}

// Engineering shear strain of an edge: (u_hi - u_lo) / h + (w_hi - w_lo) / h.
template <typename T>
__device__ __forceinline__ T shear_strain(T u_hi, T u_lo, T w_hi, T w_lo, T rh) {
  return fma(w_hi - w_lo, rh, (u_hi - u_lo) * rh);
}

// Edge shear modulus for the divergence: mean of the four cells around the edge
// (absent cells zero), doubled on a clamped wall, zero when inactive.
template <typename T>
__device__ __forceinline__ T edge_modulus(T mu0, T e00, T e10, T e01, T e11, bool active, bool wall) {
  if (!active) return T(0);
  const T m = T(0.25) * mu0 * (((e00 + e10) + e01) + e11);
  return wall ? T(2) * m : m;
}

// Residual of a face unknown: load + h^2 (normal-stress jump + two shear jumps).
template <typename T>
__device__ __forceinline__ T residual(T b, T h2, T s1, T s0, T t1, T t0, T q1, T q0) {
  return fma(h2, ((s1 - s0) + (t1 - t0)) + (q1 - q0), b);
}

template <typename T>
__device__ __forceinline__ void update(T ca, T cc, T dt, T r, T& u, T& v) {
  v = fma(cc, r, ca * v);
  u = fma(dt, v, u);
}

}  // namespace el3d
}  // namespace petto
