// 3D staggered-grid elastic sweep, streamed along z (gfx950).
//
// A workgroup owns a TX x TY column of grid positions and marches through KZ
// z-layers.  LDS holds the state and moduli of two consecutive layers (k, k+1)
// with a one-position xy halo (reflected ghosts of clamped sides filled in), the
// normal stresses and xy-shear of layer k, and the xz/yz-shear planes at z = k
// and z = k+1.  Per layer: load layer k+1, form the stresses that need it, then
// the residuals and the damped update of layer k (Eqs. 3.6, 3.9, 3.10, 3.12).
// Each state value is read from memory about once per sweep (plus the xy halo).
#include "el3d_ops.hpp"
#include "kernels.hpp"

#pragma clang fp contract(off)

namespace petto {
namespace {

constexpr int TX = 64;
constexpr int LX = TX + 3;   // halo column on each side, plus the x = nx face column
// (likewise LY = TY + 3 rows: halo rows and the y = ny face row)

template <typename T, int TY>
struct Sm3 {
  static constexpr int LY = TY + 3;
  T u[2][3][LY][LX];        // state planes (parity of the layer), with halo
  T e[2][LY][LX];           // cell moduli of the same layers
  T sxx[LY][LX], syy[LY][LX];
  T txy[LY][LX];
  T txz[2][LY][LX];         // xz shear at z = layer (parity)
  T tyz[2][LY][LX];
  double red[TX * TY / kWave];
};

__device__ __forceinline__ bool pinned3s(const uint32_t* pins, long k) {
  return pins != nullptr && ((pins[k >> 5] >> (k & 31)) & 1u);
}

// Component a at face position (i, j, k) with the reflected ghosts of clamped sides
// (one foreign axis out of range by one); zero elsewhere outside the grid.
template <typename T>
__device__ __forceinline__ T face3(const ElGeom& g, const T* __restrict__ u, int a, int i, int j, int k) {
  int id[3] = {i, j, k};
  const int n[3] = {g.nx, g.ny, g.nz};
  if (id[a] < 0 || id[a] > n[a]) return T(0);
  T sgn = T(1);
  int out = 0;
#pragma unroll
  for (int b = 0; b < 3; ++b) {
    if (b == a) continue;
    if (id[b] == -1) { out += 1; sgn = g.clamp[2 * b] ? -sgn : T(0); id[b] = 0; }
    else if (id[b] == n[b]) { out += 1; sgn = g.clamp[2 * b + 1] ? -sgn : T(0); id[b] = n[b] - 1; }
    else if (id[b] < -1 || id[b] > n[b]) { out += 2; }
  }
  if (out > 1 || sgn == T(0)) return T(0);
  return sgn * u[(long)a * g.plane + ((long)id[2] * g.py + id[1]) * g.px + id[0]];
}

// Staging of one z-layer: each thread fetches its share of the (TY+3) x (TX+3)
// plane into registers (ahead of time) and later stores it to LDS.
template <typename T, int TY>
struct Plane {
  static constexpr int LY = TY + 3;
  static constexpr int NE = (LY * LX + TX * TY - 1) / (TX * TY);
  T v[NE][4];   // u_x, u_y, u_z, modulus
};

template <typename T, int TY>
__device__ __forceinline__ void fetch_plane(const ElGeom& g, const T* __restrict__ u, const T* __restrict__ E,
                                            int i0, int j0, int k, Plane<T, TY>& P) {
  constexpr int LY = TY + 3;
#pragma unroll
  for (int e = 0; e < Plane<T, TY>::NE; ++e) {
    const int q = threadIdx.x + e * TX * TY;
    P.v[e][0] = P.v[e][1] = P.v[e][2] = P.v[e][3] = T(0);
    if (q >= LY * LX) continue;
    const int b = q / LX, a = q - b * LX;
    const int i = i0 - 1 + a, j = j0 - 1 + b;
    if (i >= 0 && i < g.nx && j >= 0 && j < g.ny && k >= 0 && k < g.nz) {
      // interior: every component's indices are in range, no ghosts
      const long p = ((long)k * g.py + j) * g.px + i;
      P.v[e][0] = u[p];
      P.v[e][1] = u[g.plane + p];
      P.v[e][2] = u[2 * g.plane + p];
      P.v[e][3] = E != nullptr ? E[((long)k * g.ny + j) * g.nx + i] : T(0);
    } else {
      P.v[e][0] = face3<T>(g, u, 0, i, j, k);
      P.v[e][1] = face3<T>(g, u, 1, i, j, k);
      P.v[e][2] = face3<T>(g, u, 2, i, j, k);
    }
  }
}

template <typename T, int TY>
__device__ __forceinline__ void store_plane(const Plane<T, TY>& P, int buf, Sm3<T, TY>& sm) {
  constexpr int LY = TY + 3;
#pragma unroll
  for (int e = 0; e < Plane<T, TY>::NE; ++e) {
    const int q = threadIdx.x + e * TX * TY;
    if (q >= LY * LX) continue;
    const int b = q / LX, a = q - b * LX;
    sm.u[buf][0][b][a] = P.v[e][0];
    sm.u[buf][1][b][a] = P.v[e][1];
    sm.u[buf][2][b][a] = P.v[e][2];
    sm.e[buf][b][a] = P.v[e][3];
  }
}

// side activity along one axis for an edge index; sets `on` on a side
__device__ __forceinline__ bool edge_ok(int idx, int n, int clo, int chi, bool& on) {
  if (idx == 0) { on = true; return clo != 0; }
  if (idx == n) { on = true; return chi != 0; }
  return idx > 0 && idx < n;
}

// xz / yz shear planes at z = kz from state planes (lower = kz-1, upper = kz).
template <typename T, int TY>
__device__ __forceinline__ void xz_yz_planes(const ElGeom& g, int i0, int j0, int kz, int lo, int up, int dst,
                                             T rh, T mu0, Sm3<T, TY>& sm) {
  constexpr int LY = TY + 3;
  for (int q = threadIdx.x; q < LY * LX; q += TX * TY) {
    const int b = q / LX, a = q - b * LX;
    const int i = i0 - 1 + a, j = j0 - 1 + b;
    T txz = T(0), tyz = T(0);
    if (a >= 1 && b >= 1) {
      // xz edge (i, j+1/2, kz): cells (i-1..i, j, kz-1..kz)
      bool on = false;
      bool act = j >= 0 && j < g.ny;
      act = act && edge_ok(i, g.nx, g.clamp[0], g.clamp[1], on);
      act = act && edge_ok(kz, g.nz, g.clamp[4], g.clamp[5], on);
      const T m = el3d::edge_modulus<T>(mu0, sm.e[lo][b][a - 1], sm.e[lo][b][a], sm.e[up][b][a - 1], sm.e[up][b][a],
                                        act, on);
      const T gam = el3d::shear_strain<T>(sm.u[up][0][b][a], sm.u[lo][0][b][a], sm.u[up][2][b][a],
                                          sm.u[up][2][b][a - 1], rh);
      txz = m * gam;
      // yz edge (i+1/2, j, kz): cells (i, j-1..j, kz-1..kz)
      bool on2 = false;
      bool act2 = i >= 0 && i < g.nx;
      act2 = act2 && edge_ok(j, g.ny, g.clamp[2], g.clamp[3], on2);
      act2 = act2 && edge_ok(kz, g.nz, g.clamp[4], g.clamp[5], on2);
      const T m2 = el3d::edge_modulus<T>(mu0, sm.e[lo][b - 1][a], sm.e[lo][b][a], sm.e[up][b - 1][a], sm.e[up][b][a],
                                         act2, on2);
      const T gam2 = el3d::shear_strain<T>(sm.u[up][1][b][a], sm.u[lo][1][b][a], sm.u[up][2][b][a],
                                           sm.u[up][2][b - 1][a], rh);
      tyz = m2 * gam2;
    }
    sm.txz[dst][b][a] = txz;
    sm.tyz[dst][b][a] = tyz;
  }
}

// sigma_zz of the own cell (i, j, k) from planes cur (k) and up (k+1)
template <typename T, int TY>
__device__ __forceinline__ T own_szz(const Sm3<T, TY>& sm, int a, int b, int cur, int up, T rh, T lam0, T mu0) {
  const T e = sm.e[cur][b][a];
  const T exx = (sm.u[cur][0][b][a + 1] - sm.u[cur][0][b][a]) * rh;
  const T eyy = (sm.u[cur][1][b + 1][a] - sm.u[cur][1][b][a]) * rh;
  const T ezz = (sm.u[up][2][b][a] - sm.u[cur][2][b][a]) * rh;
  T sxx, syy, szz;
  el3d::normal_stress<T>(e * lam0, T(2) * (e * mu0), exx, eyy, ezz, sxx, syy, szz);
  return szz;
}

// Result of one unknown: the damped update (sweep modes), the residual (kResid)
// or its FP32 rounding (kRefine); r^2 accumulated on checking modes.
template <typename T, int MODE>
__device__ __forceinline__ void finish(const ElSweep<T>& A, long gi, bool fix, T r, T un, T vn, T ca, T cc, T dt,
                                       double& acc) {
  r = fix ? T(0) : r;
  if (MODE == kSweep || MODE == kCheck) {
    if (!fix) el3d::update<T>(ca, cc, dt, r, un, vn);
    A.v[gi] = vn;
    A.uout[gi] = un;
  } else if (MODE == kResid) {
    A.v[gi] = r;
  } else {
    A.b32[gi] = (float)r;
  }
  if (MODE == kCheck || MODE == kRefine) acc += (double)r * (double)r;
}

// Padding slot of a component array: written as zero.
template <typename T, int MODE>
__device__ __forceinline__ void zero_slot(const ElSweep<T>& A, long gi) {
  if (MODE == kSweep || MODE == kCheck) A.uout[gi] = T(0);
  else if (MODE == kResid) A.v[gi] = T(0);
  else A.b32[gi] = 0.f;
}

// Tiling: x-tiles of TX positions cover i < nx, and a tile ending at i = nx - 1
// also takes the face column i = nx (only u_x lives there) through TY + 1 threads
// of its first wave; y-tiles of TY rows cover j < ny, and a tile ending at
// j = ny - 1 also takes the face row j = ny (only u_y) through its last wave;
// z-tiles of KZ layers, the last one running through layer nz.
template <typename T, int TY, int KZ, int MODE>
__global__ __launch_bounds__(TX * TY) void el3d_stream_kernel(ElGeom g, ElSweep<T> A, int tiles_x, int tiles_y,
                                                              int ntiles) {
  // the stop flag is read up front and tested after the first planes' loads are
  // issued, so the latencies overlap
  int done = 0;
  if (MODE == kSweep || MODE == kCheck || (MODE == kRefine && A.st != nullptr)) done = A.st->done;
  constexpr int LY = TY + 3;
  constexpr int XA = TX + 1;             // LDS column of the face column i = i0 + TX
  __shared__ Sm3<T, TY> sm;
  const int tile = xcd_tile(blockIdx.x, ntiles);
  const int txy = tiles_x * tiles_y;
  const int tz = tile / txy;
  const int trem = tile - tz * txy;
  const int tyi = trem / tiles_x, txi = trem - tyi * tiles_x;
  const int i0 = txi * TX, j0 = tyi * TY, k0 = tz * KZ;
  const int a = 1 + (int)(threadIdx.x % TX), b = 1 + (int)(threadIdx.x / TX);
  const int i = i0 - 1 + a, j = j0 - 1 + b;
  const int nx = g.nx, ny = g.ny, nz = g.nz;
  const long pl = g.plane;
  const T rh = T(1.0 / g.h), h2 = T(g.h * g.h);
  const T lam0 = T(g.lam0), mu0 = T(g.mu0);
  T ca = T(0), cc = T(0), dt = T(0);
  if (MODE == kSweep || MODE == kCheck) {
    ca = T(A.st->a);
    cc = T(A.st->c);
    dt = T(A.st->dt);
  }
  // face-row duty (j = ny): the last wave, lane l takes position i0 + l
  const bool yrow = j0 + TY == ny && (int)threadIdx.x / TX == TY - 1;
  const int fi = i0 + (int)(threadIdx.x % TX);
  const bool yface = yrow && fi <= nx;
  const bool yfok = yface && fi < nx;
  // face-column duty (i = nx): thread t <= TY takes row j0 + t of the column
  // (row TY only when this tile also holds the face row: the corner slot)
  const int ej = j0 + (int)threadIdx.x;
  const bool xface = i0 + TX == nx && ej <= ny && ((int)threadIdx.x < TY || ((int)threadIdx.x == TY && j0 + TY == ny));
  const bool xfok = xface && ej < ny;
  const int kend = (tz == ntiles / txy - 1) ? nz + 1 : k0 + KZ;
  // prologue: planes k0-1 (into buffer 1) and k0 (buffer 0); xz/yz shear at z = k0
  // into buffer 0; sigma_zz of the own cell at k0-1; plane k0+1 fetched ahead
  Plane<T, TY> P;
  fetch_plane<T, TY>(g, A.uin, A.E, i0, j0, k0 - 1, P);
  store_plane<T, TY>(P, 1, sm);
  fetch_plane<T, TY>(g, A.uin, A.E, i0, j0, k0, P);
  store_plane<T, TY>(P, 0, sm);
  if (done) return;   // uniform over the workgroup, before its first barrier
  __syncthreads();
  fetch_plane<T, TY>(g, A.uin, A.E, i0, j0, k0 + 1, P);
  xz_yz_planes<T, TY>(g, i0, j0, k0, 1, 0, 0, rh, mu0, sm);
  T szz_prev = own_szz<T, TY>(sm, a, b, 1, 0, rh, lam0, mu0);
  __syncthreads();
  double acc = 0.0;
  int cur = 0;
  for (int k = k0; k < kend; ++k) {
    const int up = cur ^ 1;
    // plane k+1 into LDS (its buffer was last read before the previous barrier)
    store_plane<T, TY>(P, up, sm);
    // own velocity / right-hand side of layer k
    const long p = ((long)k * g.py + j) * g.px + i;
    const bool in = i <= nx && j <= ny;
    const bool ok[3] = {in && j < ny && k < nz, in && i < nx && k < nz, in && i < nx && j < ny};
    T vv[3], bb[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      vv[c] = T(0);
      if ((MODE == kSweep || MODE == kCheck) && ok[c]) vv[c] = A.v[c * pl + p];
      bb[c] = ok[c] ? A.b[c * pl + p] : T(0);
    }
    const long pe = ((long)k * g.py + ej) * g.px + nx;
    const bool xok = xfok && k < nz;
    T vxe = T(0), bxe = T(0);
    if (xok) {
      if (MODE == kSweep || MODE == kCheck) vxe = A.v[pe];
      bxe = A.b[pe];
    }
    const long pf = ((long)k * g.py + ny) * g.px + fi;
    const bool yok = yfok && k < nz;
    T vye = T(0), bye = T(0);
    if (yok) {
      if (MODE == kSweep || MODE == kCheck) vye = A.v[pl + pf];
      bye = A.b[pl + pf];
    }
    __syncthreads();
    // fetch plane k+2 while this layer computes
    if (k + 1 < kend) fetch_plane<T, TY>(g, A.uin, A.E, i0, j0, k + 2, P);
    const T uo[3] = {sm.u[cur][0][b][a], sm.u[cur][1][b][a], sm.u[cur][2][b][a]};
    const T uxe = xok ? sm.u[cur][0][1 + threadIdx.x][XA] : T(0);
    const T uye = yok ? sm.u[cur][1][TY + 1][1 + threadIdx.x % TX] : T(0);
    // normal stresses (cells of layer k) and xy shear (layer k)
    for (int q = threadIdx.x; q < LY * LX; q += TX * TY) {
      const int bb2 = q / LX, aa = q - bb2 * LX;
      T sxx = T(0), syy = T(0), txy_ = T(0);
      if (aa + 1 < LX && bb2 + 1 < LY) {
        const T e = sm.e[cur][bb2][aa];
        const T exx = (sm.u[cur][0][bb2][aa + 1] - sm.u[cur][0][bb2][aa]) * rh;
        const T eyy = (sm.u[cur][1][bb2 + 1][aa] - sm.u[cur][1][bb2][aa]) * rh;
        const T ezz = (sm.u[up][2][bb2][aa] - sm.u[cur][2][bb2][aa]) * rh;
        T szz;
        el3d::normal_stress<T>(e * lam0, T(2) * (e * mu0), exx, eyy, ezz, sxx, syy, szz);
      }
      if (aa >= 1 && bb2 >= 1) {
        const int vi = i0 - 1 + aa, vj = j0 - 1 + bb2;
        bool on = false;
        bool act = k < nz;
        act = act && edge_ok(vi, nx, g.clamp[0], g.clamp[1], on);
        act = act && edge_ok(vj, ny, g.clamp[2], g.clamp[3], on);
        const T m = el3d::edge_modulus<T>(mu0, sm.e[cur][bb2 - 1][aa - 1], sm.e[cur][bb2 - 1][aa],
                                          sm.e[cur][bb2][aa - 1], sm.e[cur][bb2][aa], act, on);
        const T gam = el3d::shear_strain<T>(sm.u[cur][0][bb2][aa], sm.u[cur][0][bb2 - 1][aa], sm.u[cur][1][bb2][aa],
                                            sm.u[cur][1][bb2][aa - 1], rh);
        txy_ = m * gam;
      }
      sm.sxx[bb2][aa] = sxx;
      sm.syy[bb2][aa] = syy;
      sm.txy[bb2][aa] = txy_;
    }
    xz_yz_planes<T, TY>(g, i0, j0, k + 1, cur, up, up, rh, mu0, sm);
    const T szz_cur = own_szz<T, TY>(sm, a, b, cur, up, rh, lam0, mu0);
    __syncthreads();
    // residuals and update of the own position at layer k (reads stress planes only)
    if (in) {
      T rr[3];
      rr[0] = el3d::residual<T>(bb[0], h2, sm.sxx[b][a], sm.sxx[b][a - 1], sm.txy[b + 1][a], sm.txy[b][a],
                                sm.txz[up][b][a], sm.txz[cur][b][a]);
      rr[1] = el3d::residual<T>(bb[1], h2, sm.syy[b][a], sm.syy[b - 1][a], sm.txy[b][a + 1], sm.txy[b][a],
                                sm.tyz[up][b][a], sm.tyz[cur][b][a]);
      rr[2] = el3d::residual<T>(bb[2], h2, szz_cur, szz_prev, sm.txz[cur][b][a + 1], sm.txz[cur][b][a],
                                sm.tyz[cur][b + 1][a], sm.tyz[cur][b][a]);
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const long gi = c * pl + p;
        if (!ok[c]) {
          zero_slot<T, MODE>(A, gi);
          continue;
        }
        const int own = c == 0 ? i : c == 1 ? j : k;
        const int nown = c == 0 ? nx : c == 1 ? ny : nz;
        const bool fix = (own == 0 && g.fixn[2 * c]) || (own == nown && g.fixn[2 * c + 1]) || pinned3s(g.pins, gi);
        finish<T, MODE>(A, gi, fix, rr[c], uo[c], vv[c], ca, cc, dt, acc);
      }
    }
    // the face column i = nx: u_x only (u_y, u_z slots are padding)
    if (xface) {
      const int eb = 1 + (int)threadIdx.x;
      if (xok) {
        const T r = el3d::residual<T>(bxe, h2, sm.sxx[eb][XA], sm.sxx[eb][XA - 1], sm.txy[eb + 1][XA],
                                      sm.txy[eb][XA], sm.txz[up][eb][XA], sm.txz[cur][eb][XA]);
        const bool fix = g.fixn[1] || pinned3s(g.pins, pe);
        finish<T, MODE>(A, pe, fix, r, uxe, vxe, ca, cc, dt, acc);
      } else {
        zero_slot<T, MODE>(A, pe);
      }
      zero_slot<T, MODE>(A, pl + pe);
      zero_slot<T, MODE>(A, 2 * pl + pe);
    }
    // the face row j = ny: u_y only (u_x, u_z slots are padding)
    if (yface) {
      const int fa = 1 + (int)(threadIdx.x % TX), fb = TY + 1;
      if (yok) {
        const T r = el3d::residual<T>(bye, h2, sm.syy[fb][fa], sm.syy[fb - 1][fa], sm.txy[fb][fa + 1],
                                      sm.txy[fb][fa], sm.tyz[up][fb][fa], sm.tyz[cur][fb][fa]);
        const bool fix = g.fixn[3] || pinned3s(g.pins, pl + pf);
        finish<T, MODE>(A, pl + pf, fix, r, uye, vye, ca, cc, dt, acc);
      } else {
        zero_slot<T, MODE>(A, pl + pf);
      }
      zero_slot<T, MODE>(A, pf);
      zero_slot<T, MODE>(A, 2 * pl + pf);
    }
    szz_prev = szz_cur;
    cur = up;
    // the next store writes the plane read before the barrier above, and the
    // stress planes read here are rewritten only after the next barrier
  }
  if (MODE == kCheck || MODE == kRefine) {
    const double s = block_sum(acc, sm.red);
    if (threadIdx.x == 0) A.partial[tile] = s;
  }
}

// Two tilings per precision: columns of 64 x TY positions streamed through KZ
// layers.  The large one moves the fewest halo bytes; the small one gives
// small grids enough workgroups to fill the chip.
template <typename T, int V> struct Cfg3;
template <> struct Cfg3<float, 1> { static constexpr int TY = 8, KZ = 8; };
template <> struct Cfg3<float, 2> { static constexpr int TY = 4, KZ = 4; };
template <> struct Cfg3<double, 1> { static constexpr int TY = 4, KZ = 8; };
template <> struct Cfg3<double, 2> { static constexpr int TY = 4, KZ = 4; };

template <typename T, int V>
void tiles_s(const ElGeom& g, int& tx, int& ty, int& tz) {
  tx = (g.nx + TX - 1) / TX;
  ty = (g.ny + Cfg3<T, V>::TY - 1) / Cfg3<T, V>::TY;
  tz = (g.nz + Cfg3<T, V>::KZ - 1) / Cfg3<T, V>::KZ;
}

template <typename T, int V>
int count_s(const ElGeom& g) {
  int a, b, c;
  tiles_s<T, V>(g, a, b, c);
  return a * b * c;
}

template <typename T, int V, int MODE>
int launch_v(const ElGeom& g, const ElSweep<T>& a, hipStream_t s) {
  int tx, ty, tz;
  tiles_s<T, V>(g, tx, ty, tz);
  const int nt = tx * ty * tz;
  constexpr int TY = Cfg3<T, V>::TY, KZ = Cfg3<T, V>::KZ;
  hipLaunchKernelGGL((el3d_stream_kernel<T, TY, KZ, MODE>), dim3(nt), dim3(TX * TY), 0, s, g, a, tx, ty, nt);
  return nt;
}

}  // namespace

int el3d_tiles_prec(const ElGeom& g, bool fp64) {
  if (fp64) return g.tile3d == 2 ? count_s<double, 2>(g) : count_s<double, 1>(g);
  return g.tile3d == 2 ? count_s<float, 2>(g) : count_s<float, 1>(g);
}

int el3d_tiles(const ElGeom& g) {
  const int c[4] = {count_s<float, 1>(g), count_s<float, 2>(g), count_s<double, 1>(g), count_s<double, 2>(g)};
  int m = 0;
  for (int x : c) m = x > m ? x : m;
  return m;
}

int el3d_choose_tiling(const ElGeom& g, bool fp64, int ncu) {
  const int large = fp64 ? count_s<double, 1>(g) : count_s<float, 1>(g);
  return large >= 2 * ncu ? 1 : 2;
}

template <typename T, int MODE>
int launch_el3d(const ElGeom& g, const ElSweep<T>& a, hipStream_t s) {
  return g.tile3d == 2 ? launch_v<T, 2, MODE>(g, a, s) : launch_v<T, 1, MODE>(g, a, s);
}

template int launch_el3d<float, kSweep>(const ElGeom&, const ElSweep<float>&, hipStream_t);
template int launch_el3d<float, kCheck>(const ElGeom&, const ElSweep<float>&, hipStream_t);
template int launch_el3d<float, kResid>(const ElGeom&, const ElSweep<float>&, hipStream_t);
template int launch_el3d<double, kSweep>(const ElGeom&, const ElSweep<double>&, hipStream_t);
template int launch_el3d<double, kCheck>(const ElGeom&, const ElSweep<double>&, hipStream_t);
template int launch_el3d<double, kResid>(const ElGeom&, const ElSweep<double>&, hipStream_t);
template int launch_el3d<double, kRefine>(const ElGeom&, const ElSweep<double>&, hipStream_t);

}  // namespace petto
