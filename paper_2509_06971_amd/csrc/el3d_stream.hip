// 3D staggered-grid elastic sweep, streamed along z (gfx950).
//
// A workgroup owns a TX x TY column of grid positions and marches through its
// z-layers.  LDS holds the state and moduli of two consecutive layers (k, k+1)
// with a halo (reflected ghosts of clamped sides filled in), the normal stresses
// and xy-shear of layer k, and the xz/yz-shear planes at z = k and z = k+1.  Per
// layer: store layer k+1 (fetched into registers one layer ahead), form the
// stresses that need it, then the residuals and the damped update of layer k
// (Eqs. 3.6, 3.9, 3.10, 3.12).  Each state value is read from memory about once
// per sweep plus the xy halo.
//
// Everything that depends only on a staged entry's xy position (source offsets,
// ghost multipliers, edge activity) is worked out once per workgroup; a layer
// adds only layer-uniform terms, so the per-layer work is the stencil itself.
// Offsets within a layer are 32-bit and relative to each component's array.
#include <type_traits>

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

// Entry flags (one bit each, kept in a vector register: per-lane booleans held as
// scalar lane masks would exhaust the scalar registers).
enum : unsigned {
  kMe = 1u,        // the entry is a cell of the grid (modulus present)
  kNrm = 2u,       // forms normal stresses (not the last row or column)
  kShr = 4u,       // forms shear edges (not the first row or column)
  kAxy = 8u,       // xy edge active (inside the z range)
  kWxy = 16u,      // xy edge on a wall
  kAxz = 32u,      // xz edge: xy part of the activity
  kWxz = 64u,      // xz edge: on an x wall
  kAyz = 128u,     // yz edge: xy part of the activity
  kWyz = 256u,     // yz edge: on a y wall
};

// Bits of a thread's own-position word.
enum : unsigned {
  kIn = 1u,        // position inside the padded grid (i <= nx, j <= ny)
  kOkx = 2u,       // u_x exists here (below layer nz)
  kOky = 4u,       // u_y exists here (below layer nz)
  kOkz = 8u,       // u_z exists here
  kFixx = 16u,     // u_x on a side that holds it
  kFixy = 32u,     // u_y on a side that holds it
  kYface = 64u,    // takes a slot of the y = ny face row
  kYfok = 128u,    // ... where u_y exists
  kXface = 256u,   // takes a slot of the x = nx face column
  kXfok = 512u,    // ... where u_x exists
};

// What one staged LDS entry needs, worked out once per workgroup.
template <typename T>
struct Entry {
  int ox, oy, oz, oe;       // in-layer source offsets (u_x, u_y, u_z, modulus)
  T mx, my, mz;             // multipliers inside the z range: +1, -1 (reflected ghost) or 0
  T gx, gy;                 // u_x / u_y multipliers on the z-ghost layers (0 at corners)
  unsigned f;               // flags above
  int eb, ea;               // LDS row and column
  __device__ bool has(unsigned bit) const { return (f & bit) != 0u; }
};

template <typename T>
__device__ __forceinline__ void make_entry(const ElGeom& g, int q, int i0, int j0, Entry<T>& E) {
  const int nx = g.nx, ny = g.ny;
  E.eb = q / LX;
  E.ea = q - E.eb * LX;
  const int i = i0 - 1 + E.ea, j = j0 - 1 + E.eb;
  int si, sj;
  bool gh_i, gh_j;
  const int ri = reflect(i, nx, g.clamp[0], g.clamp[1], si, gh_i);
  const int rj = reflect(j, ny, g.clamp[2], g.clamp[3], sj, gh_j);
  // u_x(i, j): own axis x in [0, nx], foreign axis y
  const bool own_x = i >= 0 && i <= nx;
  E.mx = T(own_x ? rj : 0);
  E.ox = own_x ? sj * g.px + i : 0;
  E.gx = gh_j ? T(0) : E.mx;
  // u_y(i, j): own axis y in [0, ny], foreign axis x
  const bool own_y = j >= 0 && j <= ny;
  E.my = T(own_y ? ri : 0);
  E.oy = own_y ? j * g.px + si : 0;
  E.gy = gh_i ? T(0) : E.my;
  // u_z(i, j): foreign axes x and y; outside on both is a corner (zero)
  E.mz = T((gh_i && gh_j) ? 0 : ri * rj);
  E.oz = sj * g.px + si;
  // cell modulus
  const bool me = i >= 0 && i < nx && j >= 0 && j < ny;
  E.oe = me ? j * nx + i : 0;
  bool on = false;
  const bool ai = edge_ok(i, nx, g.clamp[0], g.clamp[1], on);
  const bool aj = edge_ok(j, ny, g.clamp[2], g.clamp[3], on);
  bool on2 = false;
  const bool ai2 = edge_ok(i, nx, g.clamp[0], g.clamp[1], on2);
  bool on3 = false;
  const bool aj3 = edge_ok(j, ny, g.clamp[2], g.clamp[3], on3);
  unsigned f = 0u;
  f |= me ? kMe : 0u;
  f |= (E.ea + 1 < LX) ? kNrm : 0u;
  f |= (E.ea >= 1 && E.eb >= 1) ? kShr : 0u;
  f |= (ai && aj) ? kAxy : 0u;
  f |= on ? kWxy : 0u;
  f |= (j >= 0 && j < ny && ai2) ? kAxz : 0u;
  f |= on2 ? kWxz : 0u;
  f |= (i >= 0 && i < nx && aj3) ? kAyz : 0u;
  f |= on3 ? kWyz : 0u;
  E.f = f;
}

template <typename T>
__device__ __forceinline__ T apply_mult(T m, T v) {
  return m == T(0) ? T(0) : m * v;
}

template <typename T, int TY>
struct Plane {
  static constexpr int LY = TY + 3;
  static constexpr int NE = (LY * LX + TX * TY - 1) / (TX * TY);
  T v[NE][4];   // u_x, u_y, u_z, modulus
};

// Staging of z-layer k into registers.  Layer-uniform part: the source layers
// and whether the layer is inside [0, nz), a z-ghost layer (k = -1 or nz: u_x,
// u_y reflected across a clamped z side, else zero) or beyond (zero); u_z lives
// on layers 0..nz and the modulus on 0..nz-1.
template <typename T, int TY>
__device__ __forceinline__ void fetch_plane(const ElGeom& g, const T* __restrict__ ux, const T* __restrict__ uy,
                                            const T* __restrict__ uz, const T* __restrict__ E, int S, int SE,
                                            const Entry<T> (&en)[Plane<T, TY>::NE], int k, Plane<T, TY>& P) {
  constexpr int LY = TY + 3;
  const int nz = g.nz;
  const int kxy = k < 0 ? 0 : (k >= nz ? nz - 1 : k);
  const int kzs = k < 0 ? 0 : (k > nz ? nz : k);
  const bool inside = k >= 0 && k < nz;
  const bool zghost = k == -1 || k == nz;
  const T gs = T((k == -1 ? g.clamp[4] : g.clamp[5]) ? -1 : 0);
  const bool zok = k >= 0 && k <= nz;
  const int bxy = kxy * S, bz = kzs * S, be = kxy * SE;
#pragma unroll
  for (int e = 0; e < Plane<T, TY>::NE; ++e) {
    const int q = threadIdx.x + e * TX * TY;
    if (e > 0 && q >= LY * LX) continue;
    const T vx = ux[bxy + en[e].ox];
    const T vy = uy[bxy + en[e].oy];
    const T vz = uz[bz + en[e].oz];
    const T ve = E != nullptr ? E[be + en[e].oe] : T(0);
    const T fx = inside ? en[e].mx : (zghost ? gs * en[e].gx : T(0));
    const T fy = inside ? en[e].my : (zghost ? gs * en[e].gy : T(0));
    P.v[e][0] = apply_mult(fx, vx);
    P.v[e][1] = apply_mult(fy, vy);
    P.v[e][2] = zok ? apply_mult(en[e].mz, vz) : T(0);
    P.v[e][3] = (inside && en[e].has(kMe)) ? ve : T(0);
  }
}

template <typename T, int TY>
__device__ __forceinline__ void store_plane(const Plane<T, TY>& P, const Entry<T> (&en)[Plane<T, TY>::NE], int buf,
                                            Sm3<T, TY>& sm) {
  constexpr int LY = TY + 3;
#pragma unroll
  for (int e = 0; e < Plane<T, TY>::NE; ++e) {
    const int q = threadIdx.x + e * TX * TY;
    if (e > 0 && q >= LY * LX) continue;
    sm.u[buf][0][en[e].eb][en[e].ea] = P.v[e][0];
    sm.u[buf][1][en[e].eb][en[e].ea] = P.v[e][1];
    sm.u[buf][2][en[e].eb][en[e].ea] = P.v[e][2];
    sm.e[buf][en[e].eb][en[e].ea] = P.v[e][3];
  }
}

// xz / yz shear at z = kz of one entry from state planes lo (kz-1) and up (kz);
// act_z / wall_z: the layer's part of the edge activity.
template <typename T, int TY>
__device__ __forceinline__ void xz_yz_entry(const Entry<T>& E, int lo, int up, int dst, bool act_z, bool wall_z, T rh,
                                            T mu0, Sm3<T, TY>& sm) {
  const int b = E.eb, a = E.ea;
  T txz = T(0), tyz = T(0);
  if (E.has(kShr)) {
    // xz edge (i, j+1/2, kz): cells (i-1..i, j, kz-1..kz)
    const T m = el3d::edge_modulus<T>(mu0, sm.e[lo][b][a - 1], sm.e[lo][b][a], sm.e[up][b][a - 1], sm.e[up][b][a],
                                      E.has(kAxz) && act_z, E.has(kWxz) || wall_z);
    const T gam = el3d::shear_strain<T>(sm.u[up][0][b][a], sm.u[lo][0][b][a], sm.u[up][2][b][a],
                                        sm.u[up][2][b][a - 1], rh);
    txz = m * gam;
    // yz edge (i+1/2, j, kz): cells (i, j-1..j, kz-1..kz)
    const T m2 = el3d::edge_modulus<T>(mu0, sm.e[lo][b - 1][a], sm.e[lo][b][a], sm.e[up][b - 1][a], sm.e[up][b][a],
                                       E.has(kAyz) && act_z, E.has(kWyz) || wall_z);
    const T gam2 = el3d::shear_strain<T>(sm.u[up][1][b][a], sm.u[lo][1][b][a], sm.u[up][2][b][a],
                                         sm.u[up][2][b - 1][a], rh);
    tyz = m2 * gam2;
  }
  sm.txz[dst][b][a] = txz;
  sm.tyz[dst][b][a] = tyz;
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

// Result of one unknown at index gi: the damped update (sweep modes), the
// residual (kResid) or its FP32 rounding (kRefine); r^2 summed on checking modes.
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
  constexpr int NE = Plane<T, TY>::NE;
  constexpr int LY = TY + 3;
  constexpr int XA = TX + 1;             // LDS column of the face column i = i0 + TX
  __shared__ Sm3<T, TY> sm;
  const int tile = xcd_tile(blockIdx.x, ntiles);
  const int txy = tiles_x * tiles_y;
  const int tz = tile / txy;
  const int trem = tile - tz * txy;
  const int tyi = trem / tiles_x, txi = trem - tyi * tiles_x;
  const int i0 = txi * TX, j0 = tyi * TY, k0 = tz * KZ;
  const int lane = (int)(threadIdx.x % TX);
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / TX));
  const int a = 1 + lane, b = 1 + wave;
  const int i = i0 + lane, j = j0 + wave;
  const int nx = g.nx, ny = g.ny, nz = g.nz;
  const long pl = g.plane;
  const int S = g.px * g.py;             // one layer of a component array
  const int SE = nx * ny;                // one layer of the cell arrays
  const T* ux = A.uin;
  const T* uy = A.uin + pl;
  const T* uz = A.uin + 2 * pl;
  const T rh = T(1.0 / g.h), h2 = T(g.h * g.h);
  const T lam0 = T(g.lam0), mu0 = T(g.mu0);
  T ca = T(0), cc = T(0), dt = T(0);
  if (MODE == kSweep || MODE == kCheck) {
    ca = T(A.st->a);
    cc = T(A.st->c);
    dt = T(A.st->dt);
  }
  Entry<T> en[NE];
#pragma unroll
  for (int e = 0; e < NE; ++e) {
    const int q = threadIdx.x + e * TX * TY;
    make_entry<T>(g, q < LY * LX ? q : 0, i0, j0, en[e]);
  }
  // own position: which unknowns exist and the fixed sides (z parts per layer),
  // as bits of one vector register
  unsigned own = 0u;
  {
    const bool in = i <= nx && j <= ny;
    own |= in ? kIn : 0u;
    own |= (in && j < ny) ? kOkx : 0u;
    own |= (in && i < nx) ? kOky : 0u;
    own |= (in && i < nx && j < ny) ? kOkz : 0u;
    own |= ((i == 0 && g.fixn[0]) || (i == nx && g.fixn[1])) ? kFixx : 0u;
    own |= ((j == 0 && g.fixn[2]) || (j == ny && g.fixn[3])) ? kFixy : 0u;
    // face-row duty (j = ny): the last wave, lane l takes position i0 + l
    const bool yface = j0 + TY == ny && wave == TY - 1 && i <= nx;
    own |= yface ? kYface : 0u;
    own |= (yface && i < nx) ? kYfok : 0u;
    // face-column duty (i = nx): thread t <= TY takes row j0 + t of the column
    // (row TY only when this tile also holds the face row: the corner slot)
    const int ej = j0 + (int)threadIdx.x;
    const bool xface =
        i0 + TX == nx && ej <= ny && ((int)threadIdx.x < TY || ((int)threadIdx.x == TY && j0 + TY == ny));
    own |= xface ? kXface : 0u;
    own |= (xface && ej < ny) ? kXfok : 0u;
  }
  const unsigned pl32 = (unsigned)pl;    // a component holds fewer than 2^31 values
  const unsigned S32 = (unsigned)S;
  const unsigned pxy = (unsigned)(j * g.px + i);
  const unsigned pfxy = (unsigned)(ny * g.px + i);
  const unsigned pexy = (unsigned)((j0 + (int)threadIdx.x) * g.px + nx);
  const int kend = (tz == ntiles / txy - 1) ? nz + 1 : k0 + KZ;
  // prologue: planes k0-1 (into buffer 1) and k0 (buffer 0); xz/yz shear at z = k0
  // into buffer 0; sigma_zz of the own cell at k0-1; plane k0+1 fetched ahead
  Plane<T, TY> P;
  fetch_plane<T, TY>(g, ux, uy, uz, A.E, S, SE, en, k0 - 1, P);
  store_plane<T, TY>(P, en, 1, sm);
  fetch_plane<T, TY>(g, ux, uy, uz, A.E, S, SE, en, k0, P);
  store_plane<T, TY>(P, en, 0, sm);
  if (done) return;   // uniform over the workgroup, before its first barrier
  __syncthreads();
  fetch_plane<T, TY>(g, ux, uy, uz, A.E, S, SE, en, k0 + 1, P);
  {
    bool wz = false;
    const bool az = edge_ok(k0, nz, g.clamp[4], g.clamp[5], wz);
#pragma unroll
    for (int e = 0; e < NE; ++e) {
      if (e > 0 && (int)threadIdx.x + e * TX * TY >= LY * LX) continue;
      xz_yz_entry<T, TY>(en[e], 1, 0, 0, az, wz, rh, mu0, sm);
    }
  }
  T szz_prev = own_szz<T, TY>(sm, a, b, 1, 0, rh, lam0, mu0);
  __syncthreads();
  double acc = 0.0;
  // one layer; the buffer parity is a compile-time constant (the loop below is
  // unrolled by two), so every LDS access has a constant offset
  auto layer = [&](auto parity, int k) {
    constexpr int cur = decltype(parity)::value;
    constexpr int up = cur ^ 1;
    // plane k+1 into LDS (its buffer was last read before the previous barrier)
    store_plane<T, TY>(P, en, up, sm);
    // own velocity / right-hand side of layer k (issued early, used after the stresses)
    const unsigned kS = (unsigned)k * S32;
    const unsigned p = kS + pxy;
    const bool in_z = k < nz;
    const unsigned okm = in_z ? (kOkx | kOky | kOkz) : kOkz;
    T vv[3], bb[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const bool okc = (own & okm & (kOkx << c)) != 0u;
      vv[c] = T(0);
      if ((MODE == kSweep || MODE == kCheck) && okc) vv[c] = A.v[c * pl32 + p];
      bb[c] = okc ? A.b[c * pl32 + p] : T(0);
    }
    const unsigned pe = kS + pexy;
    const bool xok = in_z && (own & kXfok) != 0u;
    T vxe = T(0), bxe = T(0);
    if (xok) {
      if (MODE == kSweep || MODE == kCheck) vxe = A.v[pe];
      bxe = A.b[pe];
    }
    const unsigned pf = kS + pfxy;
    const bool yok = in_z && (own & kYfok) != 0u;
    T vye = T(0), bye = T(0);
    if (yok) {
      if (MODE == kSweep || MODE == kCheck) vye = A.v[pl32 + pf];
      bye = A.b[pl32 + pf];
    }
    __syncthreads();
    // fetch plane k+2 while this layer computes
    if (k + 1 < kend) fetch_plane<T, TY>(g, ux, uy, uz, A.E, S, SE, en, k + 2, P);
    const T uo[3] = {sm.u[cur][0][b][a], sm.u[cur][1][b][a], sm.u[cur][2][b][a]};
    const T uxe = xok ? sm.u[cur][0][1 + threadIdx.x][XA] : T(0);
    const T uye = yok ? sm.u[cur][1][TY + 1][a] : T(0);
    // normal stresses (cells of layer k) and xy shear (layer k), then the xz/yz
    // shear planes at z = k+1
    bool wz = false;
    const bool az = edge_ok(k + 1, nz, g.clamp[4], g.clamp[5], wz);
#pragma unroll
    for (int e = 0; e < NE; ++e) {
      if (e > 0 && (int)threadIdx.x + e * TX * TY >= LY * LX) continue;
      const int eb = en[e].eb, ea = en[e].ea;
      T sxx = T(0), syy = T(0), txy_ = T(0);
      if (en[e].has(kNrm) && eb + 1 < LY) {
        const T ev = sm.e[cur][eb][ea];
        const T exx = (sm.u[cur][0][eb][ea + 1] - sm.u[cur][0][eb][ea]) * rh;
        const T eyy = (sm.u[cur][1][eb + 1][ea] - sm.u[cur][1][eb][ea]) * rh;
        const T ezz = (sm.u[up][2][eb][ea] - sm.u[cur][2][eb][ea]) * rh;
        T szz;
        el3d::normal_stress<T>(ev * lam0, T(2) * (ev * mu0), exx, eyy, ezz, sxx, syy, szz);
      }
      if (en[e].has(kShr)) {
        const T m = el3d::edge_modulus<T>(mu0, sm.e[cur][eb - 1][ea - 1], sm.e[cur][eb - 1][ea],
                                          sm.e[cur][eb][ea - 1], sm.e[cur][eb][ea], in_z && en[e].has(kAxy),
                                          en[e].has(kWxy));
        const T gam = el3d::shear_strain<T>(sm.u[cur][0][eb][ea], sm.u[cur][0][eb - 1][ea], sm.u[cur][1][eb][ea],
                                            sm.u[cur][1][eb][ea - 1], rh);
        txy_ = m * gam;
      }
      sm.sxx[eb][ea] = sxx;
      sm.syy[eb][ea] = syy;
      sm.txy[eb][ea] = txy_;
      xz_yz_entry<T, TY>(en[e], cur, up, up, az, wz, rh, mu0, sm);
    }
    const T szz_cur = own_szz<T, TY>(sm, a, b, cur, up, rh, lam0, mu0);
    __syncthreads();
    // residuals and update of the own position at layer k (reads stress planes only)
    if (own & kIn) {
      T rr[3];
      rr[0] = el3d::residual<T>(bb[0], h2, sm.sxx[b][a], sm.sxx[b][a - 1], sm.txy[b + 1][a], sm.txy[b][a],
                                sm.txz[up][b][a], sm.txz[cur][b][a]);
      rr[1] = el3d::residual<T>(bb[1], h2, sm.syy[b][a], sm.syy[b - 1][a], sm.txy[b][a + 1], sm.txy[b][a],
                                sm.tyz[up][b][a], sm.tyz[cur][b][a]);
      rr[2] = el3d::residual<T>(bb[2], h2, szz_cur, szz_prev, sm.txz[cur][b][a + 1], sm.txz[cur][b][a],
                                sm.tyz[cur][b + 1][a], sm.tyz[cur][b][a]);
      const bool fixz = (k == 0 && g.fixn[4]) || (k == nz && g.fixn[5]);
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const unsigned gi = c * pl32 + p;
        if ((own & okm & (kOkx << c)) == 0u) {
          zero_slot<T, MODE>(A, gi);
          continue;
        }
        const bool fixc = c == 0 ? (own & kFixx) != 0u : (c == 1 ? (own & kFixy) != 0u : fixz);
        finish<T, MODE>(A, gi, fixc || pinned3s(g.pins, gi), rr[c], uo[c], vv[c], ca, cc, dt, acc);
      }
    }
    // the face column i = nx: u_x only (u_y, u_z slots are padding)
    if (own & kXface) {
      const int eb = 1 + (int)threadIdx.x;
      if (xok) {
        const T r = el3d::residual<T>(bxe, h2, sm.sxx[eb][XA], sm.sxx[eb][XA - 1], sm.txy[eb + 1][XA],
                                      sm.txy[eb][XA], sm.txz[up][eb][XA], sm.txz[cur][eb][XA]);
        finish<T, MODE>(A, pe, g.fixn[1] || pinned3s(g.pins, pe), r, uxe, vxe, ca, cc, dt, acc);
      } else {
        zero_slot<T, MODE>(A, pe);
      }
      zero_slot<T, MODE>(A, pl32 + pe);
      zero_slot<T, MODE>(A, 2 * pl32 + pe);
    }
    // the face row j = ny: u_y only (u_x, u_z slots are padding)
    if (own & kYface) {
      const int fb = TY + 1;
      if (yok) {
        const T r = el3d::residual<T>(bye, h2, sm.syy[fb][a], sm.syy[fb - 1][a], sm.txy[fb][a + 1],
                                      sm.txy[fb][a], sm.tyz[up][fb][a], sm.tyz[cur][fb][a]);
        finish<T, MODE>(A, pl32 + pf, g.fixn[3] || pinned3s(g.pins, pl32 + pf), r, uye, vye, ca, cc, dt, acc);
      } else {
        zero_slot<T, MODE>(A, pl32 + pf);
      }
      zero_slot<T, MODE>(A, pf);
      zero_slot<T, MODE>(A, 2 * pl32 + pf);
    }
    szz_prev = szz_cur;
    // the next store writes the plane read before the barrier above, and the
    // stress planes read here are rewritten only after the next barrier
  };
  for (int k = k0; k < kend; k += 2) {
    layer(std::integral_constant<int, 0>(), k);
    if (k + 1 >= kend) break;
    layer(std::integral_constant<int, 1>(), k + 1);
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
