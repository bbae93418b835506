// Per-cell arithmetic of the heat sweep, shared by the one-sweep and the
// multi-sweep kernels (every rounding step spelled out, no contraction).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace petto {
namespace heat {

// Face conductance: arithmetic mean of the two cells (0 for a boundary face).
template <typename T>
__device__ __forceinline__ T face(T kc, T kn, bool exists) {
  return exists ? T(0.5) * (kc + kn) : T(0);
}

// Residual of a cell: source - sum over faces k_f (T_c - T_nb) - 2 n_D k_c T_c,
// with n_D the number of Dirichlet faces of the cell (reflected ghost T = -T_c).
template <typename T>
__device__ __forceinline__ T residual(T b, T tc, T kl, T tl, T kr, T tr, T kd, T td, T ku, T tu, T dd) {
  const T flux = fma(ku, tc - tu, fma(kd, tc - td, fma(kr, tc - tr, kl * (tc - tl))));
  return fma(-dd, tc, b - flux);
}

// Dirichlet faces of cell (i, j) from the design's side tables: [ny] low-x,
// [ny] high-x, [nx] low-y, [nx] high-y (1 = sink face).
__device__ __forceinline__ int dirichlet_count(const uint8_t* t, int nx, int ny, int i, int j) {
  int n = 0;
  if (i == 0) n += t[j];
  if (i == nx - 1) n += t[ny + j];
  if (j == 0) n += t[2 * ny + i];
  if (j == ny - 1) n += t[2 * ny + nx + i];
  return n;
}

template <typename T>
__device__ __forceinline__ void update(T ca, T cc, T dt, T r, T& u, T& v) {
  v = fma(cc, r, ca * v);
  u = fma(dt, v, u);
}

}  // namespace heat
}  // namespace petto
