// 2D staggered-grid elasticity: fused APT sweep, residual, refinement residual and
// sensitivity kernels for gfx950.
//
// One workgroup owns a 64 x 8 tile of grid positions (i, j), i in [0, nx], j in [0, ny];
// position (i, j) carries u_x(i, j) (x-face, valid for j < ny) and u_y(i, j) (y-face,
// valid for i < nx).  The tile of u and of the cell modulus is staged in LDS with a
// one-position halo, ghost values of clamped sides already reflected.  The chain is
// strain -> stress (cells: normal stresses, vertices: shear stress) -> divergence +
// load = residual r (force units) -> v <- a v + c r, u <- u + dt v (Eqs. 3.9, 3.10,
// 3.6 and the damped update of Eq. 3.12).  A wavefront owns one 64-wide row, so all
// global accesses are row-coalesced.
#include "el2d_ops.hpp"
#include "kernels.hpp"
#include "material.hpp"

// Rounding is spelled out in el2d_ops.hpp; keep the compiler from fusing further.
#pragma clang fp contract(off)

namespace petto {
namespace {

constexpr int TX = 64, TY = 8;
constexpr int LX = TX + 2, LY = TY + 2;
constexpr int RPT = TY / (kBlock / TX);   // rows per thread

template <typename T>
struct Smem {
  T ux[LY][LX];
  T uy[LY][LX];
  T E[LY][LX];
  T sxx[TY + 1][TX + 1];
  T syy[TY + 1][TX + 1];
  T tau[LY][LX];
  double red[kBlock / kWave];
};

__device__ inline bool pinned(const uint32_t* pins, long k) {
  return pins != nullptr && ((pins[k >> 5] >> (k & 31)) & 1u);
}

// Stage u (+ ghosts) and E of positions [i0-1, i0+TX] x [j0-1, j0+TY].  Every
// staged value is one load from an index inside the arrays (a ghost reads the
// value it reflects, a slot outside reads element 0) and a select: +value,
// -value (reflected ghost of a clamped side) or zero.  All loads of a thread
// are issued before the first is used, so the tile costs one memory round trip.
template <typename T>
__device__ inline void load_tile(const ElGeom& g, const T* __restrict__ u, const T* __restrict__ E,
                                 int i0, int j0, T (*sux)[LX], T (*suy)[LX], T (*sE)[LX]) {
  constexpr int NS = (LY * LX + kBlock - 1) / kBlock;
  const int nx = g.nx, ny = g.ny, px = g.px;
  const long pl = g.plane;
  T vx[NS], vy[NS], ve[NS];
  int sx[NS], sy[NS];      // +1 value, -1 reflected ghost, 0 zero
  bool se[NS];
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    const int idx0 = (int)threadIdx.x + s * kBlock;
    const int idx = idx0 < LY * LX ? idx0 : LY * LX - 1;
    const int lj = idx / LX, li = idx - lj * LX;
    const int i = i0 - 1 + li, j = j0 - 1 + lj;
    // u_x(i, j): x-face i in [0, nx], rows j in [0, ny); ghost rows -1 and ny
    long px_src = 0;
    sx[s] = 0;
    if (i >= 0 && i <= nx) {
      if (j >= 0 && j < ny) { px_src = (long)j * px + i; sx[s] = 1; }
      else if (j == -1) { px_src = i; sx[s] = g.clamp[2] ? -1 : 0; }
      else if (j == ny) { px_src = (long)(ny - 1) * px + i; sx[s] = g.clamp[3] ? -1 : 0; }
    }
    // u_y(i, j): y-face j in [0, ny], columns i in [0, nx); ghost columns -1 and nx
    long py_src = 0;
    sy[s] = 0;
    if (j >= 0 && j <= ny) {
      if (i >= 0 && i < nx) { py_src = (long)j * px + i; sy[s] = 1; }
      else if (i == -1) { py_src = (long)j * px; sy[s] = g.clamp[0] ? -1 : 0; }
      else if (i == nx) { py_src = (long)j * px + nx - 1; sy[s] = g.clamp[1] ? -1 : 0; }
    }
    se[s] = E != nullptr && i >= 0 && i < nx && j >= 0 && j < ny;
    vx[s] = u[px_src];
    vy[s] = u[pl + py_src];
    ve[s] = E != nullptr ? E[se[s] ? (long)j * nx + i : 0] : T(0);
  }
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    const int idx = (int)threadIdx.x + s * kBlock;
    if (idx >= LY * LX) continue;
    const int lj = idx / LX, li = idx - lj * LX;
    sux[lj][li] = sx[s] == 0 ? T(0) : (sx[s] < 0 ? -vx[s] : vx[s]);
    suy[lj][li] = sy[s] == 0 ? T(0) : (sy[s] < 0 ? -vy[s] : vy[s]);
    if (E != nullptr) sE[lj][li] = se[s] ? ve[s] : T(0);
  }
}

// Vertex (vi, vj) is active unless it lies on a free or roller side; 'on' reports
// whether it lies on the boundary at all.
__device__ inline bool vertex_active(const ElGeom& g, int vi, int vj, bool& on) {
  bool act = vi <= g.nx && vj <= g.ny;
  on = false;
  if (vi == 0) { act = act && g.clamp[0]; on = true; }
  if (vi == g.nx) { act = act && g.clamp[1]; on = true; }
  if (vj == 0) { act = act && g.clamp[2]; on = true; }
  if (vj == g.ny) { act = act && g.clamp[3]; on = true; }
  return act;
}

template <typename T, int MODE>
__global__ __launch_bounds__(kBlock) void el2d_kernel(ElGeom g, ElSweep<T> A, int tiles_x, int ntiles) {
  if (MODE == kSweep || MODE == kCheck || (MODE == kRefine && A.st != nullptr)) {
    if (A.st->done) return;
  }
  __shared__ Smem<T> sm;
  const int tile = xcd_tile(blockIdx.x, ntiles);
  const int tyi = tile / tiles_x, txi = tile - tyi * tiles_x;
  const int i0 = txi * TX, j0 = tyi * TY;
  const int tx = threadIdx.x & (TX - 1), ty = threadIdx.x / TX;
  const int nx = g.nx, ny = g.ny, px = g.px;
  const long pl = g.plane;
  const int i = i0 + tx;

  // Issue the per-position loads (velocity, right-hand side) before the LDS phases.
  T vx[RPT], vy[RPT], bx[RPT], by[RPT];
#pragma unroll
  for (int r = 0; r < RPT; ++r) {
    const int j = j0 + ty + r * (kBlock / TX);
    const long p = (long)j * px + i;
    const bool okx = i <= nx && j < ny;
    const bool oky = i < nx && j <= ny;
    vx[r] = vy[r] = T(0);
    if (MODE == kSweep || MODE == kCheck) {
      if (okx) vx[r] = A.v[p];
      if (oky) vy[r] = A.v[pl + p];
    }
    bx[r] = okx ? A.b[p] : T(0);
    by[r] = oky ? A.b[pl + p] : T(0);
  }

  load_tile<T>(g, A.uin, A.E, i0, j0, sm.ux, sm.uy, sm.E);
  __syncthreads();

  const T lam0 = T(g.lam0), mu0 = T(g.mu0);
  for (int idx = threadIdx.x; idx < (TY + 1) * (TX + 1); idx += kBlock) {
    const int lj = idx / (TX + 1), li = idx - lj * (TX + 1);
    const T e = sm.E[lj][li];
    const T exx = sm.ux[lj][li + 1] - sm.ux[lj][li];
    const T eyy = sm.uy[lj + 1][li] - sm.uy[lj][li];
    el2d::normal_stress<T>(e * lam0, T(2) * (e * mu0), exx, eyy, sm.sxx[lj][li], sm.syy[lj][li]);
  }
  for (int idx = threadIdx.x; idx < (TY + 1) * (TX + 1); idx += kBlock) {
    const int lj = 1 + idx / (TX + 1), li = 1 + idx % (TX + 1);
    bool on;
    const bool act = vertex_active(g, i0 - 1 + li, j0 - 1 + lj, on);
    // On a clamped wall the tangential unknown also drives the reflected ghost, so
    // its coupling to the wall vertex doubles; every free unknown a wall vertex
    // touches is such a reflected tangential one.
    const T mue = el2d::vertex_modulus<T>(mu0, sm.E[lj - 1][li - 1], sm.E[lj - 1][li], sm.E[lj][li - 1],
                                          sm.E[lj][li], act, on);
    const T gam = el2d::shear_strain<T>(sm.ux[lj][li], sm.ux[lj - 1][li], sm.uy[lj][li], sm.uy[lj][li - 1]);
    sm.tau[lj][li] = mue * gam;
  }
  __syncthreads();

  T ca = T(0), cc = T(0), dt = T(0);
  if (MODE == kSweep || MODE == kCheck) {
    ca = T(A.st->a);
    cc = T(A.st->c);
    dt = T(A.st->dt);
  }
  double acc = 0.0;
  const int li = tx + 1;
#pragma unroll
  for (int r = 0; r < RPT; ++r) {
    const int j = j0 + ty + r * (kBlock / TX);
    const int lj = ty + r * (kBlock / TX) + 1;
    if (i > nx || j > ny) continue;
    const long p = (long)j * px + i;
    // ---- x component
    if (j < ny) {
      const bool fix = (i == 0 && g.fixn[0]) || (i == nx && g.fixn[1]) || pinned(g.pins, p);
      T rx = T(0);
      if (!fix)
        rx = el2d::residual<T>(bx[r], sm.sxx[lj][li], sm.sxx[lj][li - 1], sm.tau[lj + 1][li], sm.tau[lj][li]);
      if (MODE == kSweep || MODE == kCheck) {
        T un = sm.ux[lj][li], vn = vx[r];
        if (!fix) el2d::update<T>(ca, cc, dt, rx, un, vn);
        A.v[p] = vn;
        A.uout[p] = un;
      } else if (MODE == kResid) {
        A.v[p] = rx;
      } else {
        A.b32[p] = (float)rx;
      }
      if (MODE == kCheck || MODE == kRefine) acc += (double)rx * (double)rx;
    } else {
      if (MODE == kSweep || MODE == kCheck) A.uout[p] = T(0);
      else if (MODE == kResid) A.v[p] = T(0);
      else A.b32[p] = 0.f;
    }
    // ---- y component
    const long q = pl + p;
    if (i < nx) {
      const bool fix = (j == 0 && g.fixn[2]) || (j == ny && g.fixn[3]) || pinned(g.pins, q);
      T ry = T(0);
      if (!fix)
        ry = el2d::residual<T>(by[r], sm.syy[lj][li], sm.syy[lj - 1][li], sm.tau[lj][li + 1], sm.tau[lj][li]);
      if (MODE == kSweep || MODE == kCheck) {
        T un = sm.uy[lj][li], vn = vy[r];
        if (!fix) el2d::update<T>(ca, cc, dt, ry, un, vn);
        A.v[q] = vn;
        A.uout[q] = un;
      } else if (MODE == kResid) {
        A.v[q] = ry;
      } else {
        A.b32[q] = (float)ry;
      }
      if (MODE == kCheck || MODE == kRefine) acc += (double)ry * (double)ry;
    } else {
      if (MODE == kSweep || MODE == kCheck) A.uout[q] = T(0);
      else if (MODE == kResid) A.v[q] = T(0);
      else A.b32[q] = 0.f;
    }
  }
  if (MODE == kCheck || MODE == kRefine) {
    const double s = block_sum(acc, sm.red);
    if (threadIdx.x == 0) A.partial[tile] = s;
  }
}

// ------------------------------------------------------------------------------ sensitivity

template <typename U>
struct AdjSmem {
  U ux[LY][LX];
  U uy[LY][LX];
  U wx[LY][LX];
  U wy[LY][LX];
  double red[kBlock / kWave];
};

template <typename U, typename T>
__global__ __launch_bounds__(kBlock) void el2d_adjoint_kernel(ElGeom g, ElAdjoint<U, T> A, int tiles_x,
                                                              int ntiles) {
  __shared__ AdjSmem<U> sm;
  const int tile = xcd_tile(blockIdx.x, ntiles);
  const int tyi = tile / tiles_x, txi = tile - tyi * tiles_x;
  const int i0 = txi * TX, j0 = tyi * TY;
  const int tx = threadIdx.x & (TX - 1), ty = threadIdx.x / TX;
  const int nx = g.nx, ny = g.ny, px = g.px;
  const long pl = g.plane;
  const bool same = (A.w == A.u);
  load_tile<U>(g, A.u, nullptr, i0, j0, sm.ux, sm.uy, nullptr);
  if (!same) load_tile<U>(g, A.w, nullptr, i0, j0, sm.wx, sm.wy, nullptr);
  __syncthreads();
  const double rh = 1.0 / g.h, hd = g.h * g.h;
  const double lam0 = g.lam0, mu0 = g.mu0;
  const long ncell = (long)nx * ny;
  const int i = i0 + tx, li = tx + 1;
  double fu = 0.0, en = 0.0;
#pragma unroll
  for (int r = 0; r < RPT; ++r) {
    const int j = j0 + ty + r * (kBlock / TX);
    const int lj = ty + r * (kBlock / TX) + 1;
    if (i > nx || j > ny) continue;
    const long p = (long)j * px + i;
    if (j < ny) fu += A.F[p] * (double)sm.ux[lj][li];
    if (i < nx) fu += A.F[pl + p] * (double)sm.uy[lj][li];
    if (i >= nx || j >= ny) continue;
    // cell (i, j)
    auto U_ = [&](int which, int a, int b) -> double {   // which: 0 ux 1 uy 2 wx 3 wy
      if (which == 0) return (double)sm.ux[b][a];
      if (which == 1) return (double)sm.uy[b][a];
      if (which == 2) return same ? (double)sm.ux[b][a] : (double)sm.wx[b][a];
      return same ? (double)sm.uy[b][a] : (double)sm.wy[b][a];
    };
    const double exu = (U_(0, li + 1, lj) - U_(0, li, lj)) * rh;
    const double eyu = (U_(1, li, lj + 1) - U_(1, li, lj)) * rh;
    const double exw = (U_(2, li + 1, lj) - U_(2, li, lj)) * rh;
    const double eyw = (U_(3, li, lj + 1) - U_(3, li, lj)) * rh;
    double Buu = lam0 * (exu + eyu) * (exu + eyu) + 2.0 * mu0 * (exu * exu + eyu * eyu);
    double Bwu = lam0 * (exw + eyw) * (exu + eyu) + 2.0 * mu0 * (exw * exu + eyw * eyu);
#pragma unroll
    for (int dj = 0; dj < 2; ++dj)
#pragma unroll
      for (int di = 0; di < 2; ++di) {
        bool on;
        if (!vertex_active(g, i + di, j + dj, on)) continue;
        const int a = li + di, b = lj + dj;
        const double gu = (U_(0, a, b) - U_(0, a, b - 1)) * rh + (U_(1, a, b) - U_(1, a - 1, b)) * rh;
        const double gw = (U_(2, a, b) - U_(2, a, b - 1)) * rh + (U_(3, a, b) - U_(3, a - 1, b)) * rh;
        Buu += 0.25 * mu0 * gu * gu;
        Bwu += 0.25 * mu0 * gw * gu;
      }
    Buu *= hd;
    Bwu *= hd;
    const long c = (long)j * nx + i;
    double dE[kMaxPhase];
    const double E = modulus<T>(A.phi, c, ncell, A.nphase, A.e0, A.emin, A.p, A.ep, dE);
    en += E * Buu;
    for (int m = 0; m < A.nphase; ++m) A.grad[m * ncell + c] = (T)(-dE[m] * Bwu);
  }
  const double s1 = block_sum(fu, sm.red);
  const double s2 = block_sum(en, sm.red);
  if (threadIdx.x == 0) {
    A.partial_fu[tile] = s1;
    A.partial_en[tile] = s2;
  }
}

}  // namespace

int el2d_tiles(const ElGeom& g) {
  const int tx = (g.nx + 1 + TX - 1) / TX, ty = (g.ny + 1 + TY - 1) / TY;
  return tx * ty;
}

template <typename T, int MODE>
int launch_el2d(const ElGeom& g, const ElSweep<T>& a, hipStream_t s) {
  const int tiles_x = (g.nx + 1 + TX - 1) / TX;
  const int nt = el2d_tiles(g);
  hipLaunchKernelGGL((el2d_kernel<T, MODE>), dim3(nt), dim3(kBlock), 0, s, g, a, tiles_x, nt);
  return nt;
}

template <typename U, typename T>
int launch_el2d_adjoint(const ElGeom& g, const ElAdjoint<U, T>& a, hipStream_t s) {
  const int tiles_x = (g.nx + 1 + TX - 1) / TX;
  const int nt = el2d_tiles(g);
  hipLaunchKernelGGL((el2d_adjoint_kernel<U, T>), dim3(nt), dim3(kBlock), 0, s, g, a, tiles_x, nt);
  return nt;
}

template int launch_el2d<float, kSweep>(const ElGeom&, const ElSweep<float>&, hipStream_t);
template int launch_el2d<float, kCheck>(const ElGeom&, const ElSweep<float>&, hipStream_t);
template int launch_el2d<float, kResid>(const ElGeom&, const ElSweep<float>&, hipStream_t);
template int launch_el2d<double, kSweep>(const ElGeom&, const ElSweep<double>&, hipStream_t);
template int launch_el2d<double, kCheck>(const ElGeom&, const ElSweep<double>&, hipStream_t);
template int launch_el2d<double, kResid>(const ElGeom&, const ElSweep<double>&, hipStream_t);
template int launch_el2d<double, kRefine>(const ElGeom&, const ElSweep<double>&, hipStream_t);
template int launch_el2d_adjoint<float, float>(const ElGeom&, const ElAdjoint<float, float>&, hipStream_t);
template int launch_el2d_adjoint<double, float>(const ElGeom&, const ElAdjoint<double, float>&, hipStream_t);
template int launch_el2d_adjoint<double, double>(const ElGeom&, const ElAdjoint<double, double>&, hipStream_t);

}  // namespace petto
