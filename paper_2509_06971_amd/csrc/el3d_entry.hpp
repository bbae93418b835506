// Per-position set-up shared by the 3D elastic sweep kernels: where a staged
// value comes from (in-layer byte offset of its source, folded back inside the
// grid), the multiplier that turns the loaded value into the staged one (+1
// inside, -1 for the reflected ghost of a clamped side, 0 outside), and the
// xy-position part of the shear-edge factors (0 inactive, 1, 2 on a clamped
// wall).  Worked out once per workgroup; a z-layer adds only layer-uniform terms.
#pragma once
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace petto {
namespace el3d {

// side activity along one axis for an edge index; sets `on` on a side
__device__ __forceinline__ bool edge_ok(int idx, int n, int clo, int chi, bool& on) {
  if (idx == 0) { on = true; return clo != 0; }
  if (idx == n) { on = true; return chi != 0; }
  return idx > 0 && idx < n;
}

// Reflection of a face unknown along one of its foreign axes: +1 inside [0, n),
// the clamped side's -1 (0 for other sides) one step outside, 0 further out;
// `src` is the index folded back inside, `ghost` whether idx was outside.
__device__ __forceinline__ int reflect(int idx, int n, int clo, int chi, int& src, bool& ghost) {
  ghost = !(idx >= 0 && idx < n);
  src = idx;
  if (!ghost) return 1;
  if (idx == -1) { src = 0; return clo ? -1 : 0; }
  if (idx == n) { src = n - 1; return chi ? -1 : 0; }
  src = 0;
  return 0;
}

template <typename T>
struct Entry {
  unsigned ox, oy, oz, oe;  // in-layer byte offsets of the sources (u_x, u_y, u_z, modulus)
  T mx, my, mz, me;         // multipliers on layers inside [0, nz)
  T gx, gy;                 // u_x / u_y multipliers on a z-ghost layer (0 at corners)
  T fxy, fxz, fyz;          // xy-position part of the xy, xz and yz edge factors
  int q;                    // LDS index (plane kernel) or unused
};

// Entry of grid position (i, j) (either may lie outside the grid).
template <typename T>
__device__ __forceinline__ void make_entry_at(const ElGeom& g, int i, int j, Entry<T>& E) {
  const int nx = g.nx, ny = g.ny;
  int si, sj;
  bool gh_i, gh_j;
  const int ri = reflect(i, nx, g.clamp[0], g.clamp[1], si, gh_i);
  const int rj = reflect(j, ny, g.clamp[2], g.clamp[3], sj, gh_j);
  constexpr unsigned W = sizeof(T);
  // u_x(i, j): own axis x in [0, nx], foreign axis y
  const bool own_x = i >= 0 && i <= nx;
  E.mx = T(own_x ? rj : 0);
  E.ox = (unsigned)(own_x ? sj * g.px + i : 0) * W;
  E.gx = gh_j ? T(0) : E.mx;
  // u_y(i, j): own axis y in [0, ny], foreign axis x
  const bool own_y = j >= 0 && j <= ny;
  E.my = T(own_y ? ri : 0);
  E.oy = (unsigned)(own_y ? j * g.px + si : 0) * W;
  E.gy = gh_i ? T(0) : E.my;
  // u_z(i, j): foreign axes x and y; outside on both is a corner (zero)
  E.mz = T((gh_i && gh_j) ? 0 : ri * rj);
  E.oz = (unsigned)(sj * g.px + si) * W;
  // cell modulus
  const bool me = i >= 0 && i < nx && j >= 0 && j < ny;
  E.me = T(me ? 1 : 0);
  E.oe = (unsigned)(me ? j * nx + i : 0) * W;
  bool on = false;
  const bool ai = edge_ok(i, nx, g.clamp[0], g.clamp[1], on);
  const bool aj = edge_ok(j, ny, g.clamp[2], g.clamp[3], on);
  E.fxy = T((ai && aj) ? (on ? 2 : 1) : 0);
  bool onx = false;
  const bool axz = j >= 0 && j < ny && edge_ok(i, nx, g.clamp[0], g.clamp[1], onx);
  E.fxz = T(axz ? (onx ? 2 : 1) : 0);
  bool ony = false;
  const bool ayz = i >= 0 && i < nx && edge_ok(j, ny, g.clamp[2], g.clamp[3], ony);
  E.fyz = T(ayz ? (ony ? 2 : 1) : 0);
  E.q = 0;
}

// Element access at a byte offset from a workgroup-uniform base: the address is
// a scalar base plus a 32-bit vector offset (no per-lane 64-bit arithmetic).
// (The offset passes through an empty asm so that its zero extension is formed
// beside the access, where instruction selection can fold it into the
// scalar-base form, rather than hoisted out of the layer loop as a 64-bit value.)
template <typename T>
__device__ __forceinline__ T ldo(const T* __restrict__ base, unsigned off) {
  asm volatile("" : "+v"(off));
  return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + off);
}
template <typename T>
__device__ __forceinline__ void sto(T* __restrict__ base, unsigned off, T v) {
  asm volatile("" : "+v"(off));
  *reinterpret_cast<T*>(reinterpret_cast<char*>(base) + off) = v;
}

}  // namespace el3d
}  // namespace petto
