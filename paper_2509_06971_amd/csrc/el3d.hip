// 3D staggered-grid elasticity: the sensitivity kernel (per-cell bilinear energy
// of the normal strains at cells and the engineering shear strains on the xy-,
// xz- and yz-edges, Eqs. 3.9-3.10 in three dimensions), with compliance partials.
// The sweep kernels live in el3d_stream.hip.
//
// A workgroup owns TX x TY x TZ grid positions; position (i, j, k) carries u_x, u_y,
// u_z on the faces normal to x, y, z.  The halo tile of u (ghosts of clamped sides
// reflected) sits in LDS.
#include "kernels.hpp"
#include "material.hpp"

namespace petto {
namespace {

template <typename T> struct Tile;
template <> struct Tile<float> { static constexpr int TX = 64, TY = 4, TZ = 2; };
template <> struct Tile<double> { static constexpr int TX = 64, TY = 2, TZ = 2; };

template <typename T>
struct Dims {
  static constexpr int TX = Tile<T>::TX, TY = Tile<T>::TY, TZ = Tile<T>::TZ;
  static constexpr int LX = TX + 2, LY = TY + 2, LZ = TZ + 2;
  static constexpr int NH = LX * LY * LZ;                       // halo tile
  static constexpr int NC = (TX + 1) * (TY + 1) * (TZ + 1);      // cells [0,TX]x[0,TY]x[0,TZ]
  // shear edges: xy li,lj in [1,TX+1]x[1,TY+1], lk in [1,TZ]
  static constexpr int NXY = (TX + 1) * (TY + 1) * TZ;
  // xz: li in [1,TX+1], lj in [1,TY], lk in [1,TZ+1]
  static constexpr int NXZ = (TX + 1) * TY * (TZ + 1);
  // yz: li in [1,TX], lj in [1,TY+1], lk in [1,TZ+1]
  static constexpr int NYZ = TX * (TY + 1) * (TZ + 1);
  static constexpr int NPOS = TX * TY * TZ;
  static constexpr int RPT = NPOS / kBlock;
};

template <typename T>
__device__ inline int H(int li, int lj, int lk) {
  return (lk * Dims<T>::LY + lj) * Dims<T>::LX + li;
}
// Value of component `a` at face position (i, j, k) including reflected ghosts.
template <typename T>
__device__ inline T face_value(const ElGeom& g, const T* __restrict__ u, int a, int i, int j, int k) {
  const int n[3] = {g.nx, g.ny, g.nz};
  const int idx[3] = {i, j, k};
  // own axis must be in range
  if (idx[a] < 0 || idx[a] > n[a]) return T(0);
  int src[3] = {i, j, k};
  bool neg = false;
  int ghosts = 0;
  for (int b = 0; b < 3; ++b) {
    if (b == a) continue;
    if (idx[b] >= 0 && idx[b] < n[b]) continue;
    if (idx[b] == -1 && g.clamp[2 * b]) { src[b] = 0; neg = !neg; ++ghosts; continue; }
    if (idx[b] == n[b] && g.clamp[2 * b + 1]) { src[b] = n[b] - 1; neg = !neg; ++ghosts; continue; }
    return T(0);
  }
  if (ghosts > 1) return T(0);   // edge-corner ghosts are never used by an active edge
  const T val = u[(long)a * g.plane + ((long)src[2] * g.py + src[1]) * g.px + src[0]];
  return neg ? -val : val;
}

template <typename T>
__device__ inline void load_tile3(const ElGeom& g, const T* __restrict__ u, const T* __restrict__ E,
                                  int i0, int j0, int k0, T* sux, T* suy, T* suz, T* sE) {
  using D = Dims<T>;
  for (int idx = threadIdx.x; idx < D::NH; idx += kBlock) {
    const int lk = idx / (D::LX * D::LY);
    const int rem = idx - lk * D::LX * D::LY;
    const int lj = rem / D::LX, li = rem - lj * D::LX;
    const int i = i0 - 1 + li, j = j0 - 1 + lj, k = k0 - 1 + lk;
    sux[idx] = face_value<T>(g, u, 0, i, j, k);
    suy[idx] = face_value<T>(g, u, 1, i, j, k);
    suz[idx] = face_value<T>(g, u, 2, i, j, k);
    if (sE != nullptr) {
      T e = T(0);
      if (i >= 0 && i < g.nx && j >= 0 && j < g.ny && k >= 0 && k < g.nz)
        e = E[((long)k * g.ny + j) * g.nx + i];
      sE[idx] = e;
    }
  }
}

// Activity of an index along an axis for an edge: interior always, on a side only
// if that side is clamped.  Sets `on` when the index lies on a side.
__device__ inline bool axis_ok(int idx, int n, int clo, int chi, bool& on) {
  if (idx == 0) { on = true; return clo != 0; }
  if (idx == n) { on = true; return chi != 0; }
  return true;
}

// ------------------------------------------------------------------------------ sensitivity

template <typename U>
struct AdjSmem3 {
  U ux[Dims<U>::NH], uy[Dims<U>::NH], uz[Dims<U>::NH];
  U wx[Dims<U>::NH], wy[Dims<U>::NH], wz[Dims<U>::NH];
  double red[kBlock / kWave];
};

template <typename U, typename T>
__global__ __launch_bounds__(kBlock) void el3d_adjoint_kernel(ElGeom g, ElAdjoint<U, T> A, int tiles_x,
                                                              int tiles_y, int ntiles) {
  using D = Dims<U>;
  __shared__ AdjSmem3<U> sm;
  const int tile = xcd_tile(blockIdx.x, ntiles);
  const int tz = tile / (tiles_x * tiles_y);
  const int trem = tile - tz * tiles_x * tiles_y;
  const int tyi = trem / tiles_x, txi = trem - tyi * tiles_x;
  const int i0 = txi * D::TX, j0 = tyi * D::TY, k0 = tz * D::TZ;
  const int nx = g.nx, ny = g.ny, nz = g.nz;
  const long pl = g.plane;
  const bool same = (A.w == A.u);
  load_tile3<U>(g, A.u, nullptr, i0, j0, k0, sm.ux, sm.uy, sm.uz, nullptr);
  if (!same) load_tile3<U>(g, A.w, nullptr, i0, j0, k0, sm.wx, sm.wy, sm.wz, nullptr);
  __syncthreads();
  const U* wx = same ? sm.ux : sm.wx;
  const U* wy = same ? sm.uy : sm.wy;
  const U* wz = same ? sm.uz : sm.wz;
  const double rh = 1.0 / g.h, hd = g.h * g.h * g.h;
  const double lam0 = g.lam0, mu0 = g.mu0;
  const long ncell = (long)nx * ny * nz;
  double fu = 0.0, en = 0.0;
  for (int r = 0; r < D::RPT; ++r) {
    const int q = threadIdx.x + r * kBlock;
    const int pi = q % D::TX, pj = (q / D::TX) % D::TY, pk = q / (D::TX * D::TY);
    const int i = i0 + pi, j = j0 + pj, k = k0 + pk;
    if (i > nx || j > ny || k > nz) continue;
    const int li = pi + 1, lj = pj + 1, lk = pk + 1;
    const long p = ((long)k * g.py + j) * g.px + i;
    const int hc = H<U>(li, lj, lk);
    if (j < ny && k < nz) fu += A.F[p] * (double)sm.ux[hc];
    if (i < nx && k < nz) fu += A.F[pl + p] * (double)sm.uy[hc];
    if (i < nx && j < ny) fu += A.F[2 * pl + p] * (double)sm.uz[hc];
    if (i >= nx || j >= ny || k >= nz) continue;
    const double exu = ((double)sm.ux[H<U>(li + 1, lj, lk)] - (double)sm.ux[hc]) * rh;
    const double eyu = ((double)sm.uy[H<U>(li, lj + 1, lk)] - (double)sm.uy[hc]) * rh;
    const double ezu = ((double)sm.uz[H<U>(li, lj, lk + 1)] - (double)sm.uz[hc]) * rh;
    const double exw = ((double)wx[H<U>(li + 1, lj, lk)] - (double)wx[hc]) * rh;
    const double eyw = ((double)wy[H<U>(li, lj + 1, lk)] - (double)wy[hc]) * rh;
    const double ezw = ((double)wz[H<U>(li, lj, lk + 1)] - (double)wz[hc]) * rh;
    const double tu = exu + eyu + ezu, tw = exw + eyw + ezw;
    double Buu = lam0 * tu * tu + 2.0 * mu0 * (exu * exu + eyu * eyu + ezu * ezu);
    double Bwu = lam0 * tw * tu + 2.0 * mu0 * (exw * exu + eyw * eyu + ezw * ezu);
    for (int d1 = 0; d1 < 2; ++d1)
      for (int d0 = 0; d0 < 2; ++d0) {
        bool on = false;
        // xy edge (i+d0, j+d1, k)
        {
          const int vi = i + d0, vj = j + d1;
          if (axis_ok(vi, nx, g.clamp[0], g.clamp[1], on) && axis_ok(vj, ny, g.clamp[2], g.clamp[3], on)) {
            const int a = li + d0, b = lj + d1;
            const double gu = ((double)sm.ux[H<U>(a, b, lk)] - (double)sm.ux[H<U>(a, b - 1, lk)]) * rh +
                              ((double)sm.uy[H<U>(a, b, lk)] - (double)sm.uy[H<U>(a - 1, b, lk)]) * rh;
            const double gw = ((double)wx[H<U>(a, b, lk)] - (double)wx[H<U>(a, b - 1, lk)]) * rh +
                              ((double)wy[H<U>(a, b, lk)] - (double)wy[H<U>(a - 1, b, lk)]) * rh;
            Buu += 0.25 * mu0 * gu * gu;
            Bwu += 0.25 * mu0 * gw * gu;
          }
        }
        // xz edge (i+d0, j, k+d1)
        {
          const int vi = i + d0, vk = k + d1;
          if (axis_ok(vi, nx, g.clamp[0], g.clamp[1], on) && axis_ok(vk, nz, g.clamp[4], g.clamp[5], on)) {
            const int a = li + d0, c = lk + d1;
            const double gu = ((double)sm.ux[H<U>(a, lj, c)] - (double)sm.ux[H<U>(a, lj, c - 1)]) * rh +
                              ((double)sm.uz[H<U>(a, lj, c)] - (double)sm.uz[H<U>(a - 1, lj, c)]) * rh;
            const double gw = ((double)wx[H<U>(a, lj, c)] - (double)wx[H<U>(a, lj, c - 1)]) * rh +
                              ((double)wz[H<U>(a, lj, c)] - (double)wz[H<U>(a - 1, lj, c)]) * rh;
            Buu += 0.25 * mu0 * gu * gu;
            Bwu += 0.25 * mu0 * gw * gu;
          }
        }
        // yz edge (i, j+d0, k+d1)
        {
          const int vj = j + d0, vk = k + d1;
          if (axis_ok(vj, ny, g.clamp[2], g.clamp[3], on) && axis_ok(vk, nz, g.clamp[4], g.clamp[5], on)) {
            const int b = lj + d0, c = lk + d1;
            const double gu = ((double)sm.uy[H<U>(li, b, c)] - (double)sm.uy[H<U>(li, b, c - 1)]) * rh +
                              ((double)sm.uz[H<U>(li, b, c)] - (double)sm.uz[H<U>(li, b - 1, c)]) * rh;
            const double gw = ((double)wy[H<U>(li, b, c)] - (double)wy[H<U>(li, b, c - 1)]) * rh +
                              ((double)wz[H<U>(li, b, c)] - (double)wz[H<U>(li, b - 1, c)]) * rh;
            Buu += 0.25 * mu0 * gu * gu;
            Bwu += 0.25 * mu0 * gw * gu;
          }
        }
      }
    Buu *= hd;
    Bwu *= hd;
    const long c = ((long)k * ny + j) * nx + i;
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

template <typename T>
void tiles3(const ElGeom& g, int& tx, int& ty, int& tz) {
  using D = Dims<T>;
  tx = (g.nx + 1 + D::TX - 1) / D::TX;
  ty = (g.ny + 1 + D::TY - 1) / D::TY;
  tz = (g.nz + 1 + D::TZ - 1) / D::TZ;
}

}  // namespace

template <typename U, typename T>
int launch_el3d_adjoint(const ElGeom& g, const ElAdjoint<U, T>& a, hipStream_t s) {
  int tx, ty, tz;
  tiles3<U>(g, tx, ty, tz);
  const int nt = tx * ty * tz;
  hipLaunchKernelGGL((el3d_adjoint_kernel<U, T>), dim3(nt), dim3(kBlock), 0, s, g, a, tx, ty, nt);
  return nt;
}

int el3d_adjoint_tiles(const ElGeom& g) {
  int ax, ay, az, bx, by, bz;
  tiles3<float>(g, ax, ay, az);
  tiles3<double>(g, bx, by, bz);
  const int a = ax * ay * az, b = bx * by * bz;
  return a > b ? a : b;
}

template int launch_el3d_adjoint<float, float>(const ElGeom&, const ElAdjoint<float, float>&, hipStream_t);
template int launch_el3d_adjoint<double, float>(const ElGeom&, const ElAdjoint<double, float>&, hipStream_t);
template int launch_el3d_adjoint<double, double>(const ElGeom&, const ElAdjoint<double, double>&, hipStream_t);

}  // namespace petto
