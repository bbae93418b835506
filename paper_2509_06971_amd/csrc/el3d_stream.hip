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
  T lead[LX];               // the first staged row's reads one row up land here (never used)
  T u[2][3][LY][LX];        // state planes (parity of the layer), with halo
  T e[2][LY][LX];           // cell moduli of the same layers
  T sxx[LY][LX], syy[LY][LX], szz[LY][LX];
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
// The same for an offset that only this access reads: the asm acts on the
// variable in place (no copy), and the access takes it as it is.
__device__ __forceinline__ void opaque(unsigned& x) { asm volatile("" : "+v"(x)); }
template <typename T>
__device__ __forceinline__ T ldr(const T* __restrict__ base, unsigned off) {
  return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + off);
}

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

// What one staged LDS entry needs, worked out once per workgroup.  The
// multipliers are +1, -1 (reflected ghost of a clamped side) or 0; the edge
// factors 0 (inactive), 1, or 2 (on a clamped wall), so that multiplying by
// them is exact.
template <typename T>
struct Entry {
  unsigned ox, oy, oz, oe;  // in-layer byte offsets of the sources (u_x, u_y, u_z, modulus)
  T mx, my, mz, me;         // multipliers on layers inside [0, nz)
  T gx, gy;                 // u_x / u_y multipliers on a z-ghost layer (0 at corners)
  T fxy, fxz, fyz;          // xy-position part of the xy, xz and yz edge factors
  int q;                    // LDS index (row * LX + column)
};

template <typename T>
__device__ __forceinline__ void make_entry(const ElGeom& g, int q, int i0, int j0, Entry<T>& E) {
  const int nx = g.nx, ny = g.ny;
  const int eb = q / LX;
  const int ea = q - eb * LX;
  E.q = q;
  const int i = i0 - 1 + ea, j = j0 - 1 + eb;
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
}

template <typename T, int TY>
struct Plane {
  static constexpr int LY = TY + 3;
  static constexpr int NE = (LY * LX + TX * TY - 1) / (TX * TY);
  T v[NE][4];   // u_x, u_y, u_z, modulus as loaded (multipliers applied when stored)
};

// Whether the wave of this thread has staged entry e (uniform over the wave: a
// wave past the staged count skips it; lanes of the boundary wave past the count
// repeat the last entry).
template <int TY>
__device__ __forceinline__ bool wave_has_entry(int e) {
  constexpr int LY = TY + 3;
  if (e == 0) return true;
  const int w0 = __builtin_amdgcn_readfirstlane((int)(threadIdx.x & ~(unsigned)(kWave - 1)));
  return w0 + e * TX * TY < LY * LX;
}

// Issue the loads of z-layer k (source layers clamped into the arrays; what a
// layer outside the grid holds is settled by the multipliers when stored).
template <typename T, int TY>
__device__ __forceinline__ void fetch_plane(const ElGeom& g, const T* __restrict__ ux, const T* __restrict__ uy,
                                            const T* __restrict__ uz, const T* __restrict__ E, long S, long SE,
                                            Entry<T> (&en)[Plane<T, TY>::NE], int k, Plane<T, TY>& P) {
  const int nz = g.nz;
  const int kxy = k < 0 ? 0 : (k >= nz ? nz - 1 : k);
  const int kzs = k < 0 ? 0 : (k > nz ? nz : k);
  const T* bx = ux + kxy * S;
  const T* by = uy + kxy * S;
  const T* bz = uz + kzs * S;
  const T* be = E + kxy * SE;
#pragma unroll
  for (int e = 0; e < Plane<T, TY>::NE; ++e) {
    if (!wave_has_entry<TY>(e)) continue;
    opaque(en[e].ox);
    opaque(en[e].oy);
    opaque(en[e].oz);
    opaque(en[e].oe);
    P.v[e][0] = ldr(bx, en[e].ox);
    P.v[e][1] = ldr(by, en[e].oy);
    P.v[e][2] = ldr(bz, en[e].oz);
    P.v[e][3] = ldr(be, en[e].oe);
  }
}

// Store z-layer k into LDS buffer buf.  Inside [0, nz) the xy multipliers
// apply; a z-ghost layer (k = -1 or nz) holds u_x, u_y reflected across a
// clamped z side (else zero); u_z lives on layers 0..nz and the modulus on
// 0..nz-1; layers further out are zero.
template <typename T, int TY>
__device__ __forceinline__ void store_plane(const ElGeom& g, const Plane<T, TY>& P,
                                            const Entry<T> (&en)[Plane<T, TY>::NE], int k, int buf,
                                            Sm3<T, TY>& sm) {
  const int nz = g.nz;
  T* U0 = &sm.u[buf][0][0][0];
  T* U1 = &sm.u[buf][1][0][0];
  T* U2 = &sm.u[buf][2][0][0];
  T* EE = &sm.e[buf][0][0];
  if (k >= 0 && k < nz) {
#pragma unroll
    for (int e = 0; e < Plane<T, TY>::NE; ++e) {
      if (!wave_has_entry<TY>(e)) continue;
      const int q = en[e].q;
      U0[q] = en[e].mx * P.v[e][0];
      U1[q] = en[e].my * P.v[e][1];
      U2[q] = en[e].mz * P.v[e][2];
      EE[q] = en[e].me * P.v[e][3];
    }
  } else {
    const T gs = T(((k == -1 && g.clamp[4]) || (k == nz && g.clamp[5])) ? -1 : 0);
    const T sz = T(k >= 0 && k <= nz ? 1 : 0);
#pragma unroll
    for (int e = 0; e < Plane<T, TY>::NE; ++e) {
      if (!wave_has_entry<TY>(e)) continue;
      const int q = en[e].q;
      U0[q] = (gs * en[e].gx) * P.v[e][0];
      U1[q] = (gs * en[e].gy) * P.v[e][1];
      U2[q] = (sz * en[e].mz) * P.v[e][2];
      EE[q] = T(0);
    }
  }
}

// xz / yz shear at z = kz of one entry from state planes lo (kz-1) and up (kz)
// into buffer dst.  c25 is mu0 / 4, or 0 when the z part of the edge is
// inactive; s1 is 2 on a z wall, else 1 (the factor min(f s1, 2) then doubles
// an edge on any wall).
template <typename T, int TY>
__device__ __forceinline__ void xz_yz_entry(const Entry<T>& E, int lo, int up, int dst, T c25, T s1, T rh,
                                            Sm3<T, TY>& sm) {
  const int q = E.q;
  const T* El = &sm.e[lo][0][0];
  const T* Eu = &sm.e[up][0][0];
  const T fxz = fmin(E.fxz * s1, T(2));
  const T fyz = fmin(E.fyz * s1, T(2));
  // xz edge (i, j+1/2, kz): cells (i-1..i, j, kz-1..kz)
  const T m = (c25 * (((El[q - 1] + El[q]) + Eu[q - 1]) + Eu[q])) * fxz;
  const T gam = el3d::shear_strain<T>((&sm.u[up][0][0][0])[q], (&sm.u[lo][0][0][0])[q], (&sm.u[up][2][0][0])[q],
                                      (&sm.u[up][2][0][0])[q - 1], rh);
  // yz edge (i+1/2, j, kz): cells (i, j-1..j, kz-1..kz)
  const T m2 = (c25 * (((El[q - LX] + El[q]) + Eu[q - LX]) + Eu[q])) * fyz;
  const T gam2 = el3d::shear_strain<T>((&sm.u[up][1][0][0])[q], (&sm.u[lo][1][0][0])[q], (&sm.u[up][2][0][0])[q],
                                       (&sm.u[up][2][0][0])[q - LX], rh);
  (&sm.txz[dst][0][0])[q] = m * gam;
  (&sm.tyz[dst][0][0])[q] = m2 * gam2;
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
// or its FP32 rounding (kRefine), written at byte offset off from the layer's
// component bases; r^2 summed on checking modes.
template <typename T, int MODE>
struct Out {
  T* v;        // velocity (sweep modes) or residual (kResid)
  T* u;        // state written (sweep modes)
  float* r32;  // kRefine
};

template <typename T, int MODE>
__device__ __forceinline__ void finish(const Out<T, MODE>& o, unsigned off, bool fix, T r, T un, T vn, T ca, T cc,
                                       T dt, double& acc) {
  r = fix ? T(0) : r;
  if (MODE == kSweep || MODE == kCheck) {
    if (!fix) el3d::update<T>(ca, cc, dt, r, un, vn);
    sto(o.v, off, vn);
    sto(o.u, off, un);
  } else if (MODE == kResid) {
    sto(o.v, off, r);
  } else {
    sto(o.r32, off / (unsigned)(sizeof(T) / sizeof(float)), (float)r);
  }
  if (MODE == kCheck || MODE == kRefine) acc += (double)r * (double)r;
}

// Padding slot of a component array: written as zero.
template <typename T, int MODE>
__device__ __forceinline__ void zero_slot(const Out<T, MODE>& o, unsigned off) {
  if (MODE == kSweep || MODE == kCheck) sto(o.u, off, T(0));
  else if (MODE == kResid) sto(o.v, off, T(0));
  else sto(o.r32, off / (unsigned)(sizeof(T) / sizeof(float)), 0.f);
}

// Tiling: x-tiles of TX positions cover i < nx, and a tile ending at i = nx - 1
// also takes the face column i = nx (only u_x lives there) through TY + 1 threads
// of its first wave; y-tiles of TY rows cover j < ny, and a tile ending at
// j = ny - 1 also takes the face row j = ny (only u_y) through its last wave;
// z-tiles of KZ layers, the last one also finishing the top layer nz (only u_z)
// in a short epilogue.
template <typename T, int TY, int KZ, int MODE>
__global__ __launch_bounds__(TX * TY, 4) void el3d_stream_kernel(ElGeom g, ElSweep<T> A, int tiles_x, int tiles_y,
                                                              int ntiles) {
  // the stop flag is read up front and tested after the first planes' loads are
  // issued, so the latencies overlap
  int done = 0;
  if (MODE == kSweep || MODE == kCheck || (MODE == kRefine && A.st != nullptr)) done = A.st->done;
  constexpr int NE = Plane<T, TY>::NE;
  constexpr int LY = TY + 3;
  constexpr int XA = TX + 1;             // LDS column of the face column i = i0 + TX
  constexpr unsigned W = sizeof(T);
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
  const long S = (long)g.px * g.py;      // one layer of a component array
  const long SE = (long)nx * ny;         // one layer of the cell arrays
  const T* ux = A.uin;
  const T* uy = A.uin + pl;
  const T* uz = A.uin + 2 * pl;
  const T rh = T(1.0 / g.h), h2 = T(g.h * g.h);
  const T lam0 = T(g.lam0), mu0 = T(g.mu0);
  const T c25 = T(0.25) * mu0;
  T ca = T(0), cc = T(0), dt = T(0);
  if (MODE == kSweep || MODE == kCheck) {
    ca = T(A.st->a);
    cc = T(A.st->c);
    dt = T(A.st->dt);
  }
  Entry<T> en[NE];
#pragma unroll
  for (int e = 0; e < NE; ++e) {
    const int q = (int)threadIdx.x + e * TX * TY;
    make_entry<T>(g, q < LY * LX ? q : LY * LX - 1, i0, j0, en[e]);
  }
  // own position: which unknowns exist and the fixed sides (z parts per layer),
  // as bits of one vector register
  unsigned own = 0u;
  bool plain;                            // every lane: all three unknowns, none held
  {
    const bool in = i <= nx && j <= ny;
    own |= in ? kIn : 0u;
    own |= (in && j < ny) ? kOkx : 0u;
    own |= (in && i < nx) ? kOky : 0u;
    own |= (in && i < nx && j < ny) ? kOkz : 0u;
    const bool fx = (i == 0 && g.fixn[0]) || (i == nx && g.fixn[1]);
    const bool fy = (j == 0 && g.fixn[2]) || (j == ny && g.fixn[3]);
    own |= fx ? kFixx : 0u;
    own |= fy ? kFixy : 0u;
    plain = __builtin_amdgcn_ballot_w64(!(i < nx && j < ny) || fx || fy) == 0;
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
  const bool edge_duty = (i0 + TX == nx && wave == 0) || (j0 + TY == ny && wave == TY - 1);
  plain = plain && g.pins == nullptr;
  // in-layer byte offsets of the own position (a valid slot for every lane, so the
  // loads need no guard), of the face-row slot and of the face-column slot
  const unsigned po = (own & kIn) ? (unsigned)(j * g.px + i) * W : 0u;
  const unsigned pfo = (own & kYface) ? (unsigned)(ny * g.px + i) * W : 0u;
  const unsigned peo = (own & kXface) ? (unsigned)((j0 + (int)threadIdx.x) * g.px + nx) * W : 0u;
  // LDS indices of the face-column and face-row slots (a valid index for every lane)
  const int qxe = (own & kXface) ? (1 + (int)threadIdx.x) * LX + XA : 0;
  const int qye = (own & kYface) ? (TY + 1) * LX + a : 0;
  const bool top_tile = tz == ntiles / txy - 1;
  const int kend = top_tile ? nz : k0 + KZ;
  // prologue: planes k0-1 (into buffer 1) and k0 (buffer 0); xz/yz shear at z = k0
  // into buffer 0; sigma_zz of the own cell at k0-1; plane k0+1 fetched ahead
  // (the loads of all three planes are issued before the first wait, so the
  // prologue costs one memory round trip)
  Plane<T, TY> P, Q;
  fetch_plane<T, TY>(g, ux, uy, uz, A.E, S, SE, en, k0 - 1, P);
  fetch_plane<T, TY>(g, ux, uy, uz, A.E, S, SE, en, k0, Q);
  {
    Plane<T, TY> R;
    fetch_plane<T, TY>(g, ux, uy, uz, A.E, S, SE, en, k0 + 1, R);
    store_plane<T, TY>(g, P, en, k0 - 1, 1, sm);
    store_plane<T, TY>(g, Q, en, k0, 0, sm);
    P = R;
  }
  if (done) return;   // uniform over the workgroup, before its first barrier
  __syncthreads();
  {
    bool wz = false;
    const bool az = edge_ok(k0, nz, g.clamp[4], g.clamp[5], wz);
#pragma unroll
    for (int e = 0; e < NE; ++e) {
      if (!wave_has_entry<TY>(e)) continue;
      xz_yz_entry<T, TY>(en[e], 1, 0, 0, az ? c25 : T(0), wz ? T(2) : T(1), rh, sm);
    }
  }
  T szz_prev = own_szz<T, TY>(sm, a, b, 1, 0, rh, lam0, mu0);
  __syncthreads();
  double acc = 0.0;
  const int qo = b * LX + a;
  // one layer; the buffer parity is a compile-time constant (the loop below is
  // unrolled by two), so every LDS access has a constant offset
  auto layer = [&](auto parity, auto fetch, int k) {
    constexpr int cur = decltype(parity)::value;
    constexpr int up = cur ^ 1;
    constexpr bool FETCH = decltype(fetch)::value;
    // plane k+1 into LDS (its buffer was last read before the previous barrier)
    store_plane<T, TY>(g, P, en, k + 1, up, sm);
    // own velocity / right-hand side of layer k (issued early, used after the stresses)
    const long kS = k * S;
    const T* vb = A.v + kS;
    const T* bb = A.b + kS;
    T vv[3], bv[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      vv[c] = T(0);
      if (MODE == kSweep || MODE == kCheck) vv[c] = ldo(vb + c * pl, po);
      bv[c] = ldo(bb + c * pl, po);
    }
    T vxe = T(0), bxe = T(0), vye = T(0), bye = T(0);
    if (edge_duty) {
      if (MODE == kSweep || MODE == kCheck) {
        vxe = ldo(vb, peo);
        vye = ldo(vb + pl, pfo);
      }
      bxe = ldo(bb, peo);
      bye = ldo(bb + pl, pfo);
    }
    __syncthreads();
    // fetch plane k+2 while this layer computes
    if (FETCH) fetch_plane<T, TY>(g, ux, uy, uz, A.E, S, SE, en, k + 2, P);
    const T uo[3] = {(&sm.u[cur][0][0][0])[qo], (&sm.u[cur][1][0][0])[qo], (&sm.u[cur][2][0][0])[qo]};
    T uxe = T(0), uye = T(0);
    if (edge_duty) {
      uxe = (&sm.u[cur][0][0][0])[qxe];
      uye = (&sm.u[cur][1][0][0])[qye];
    }
    // normal stresses (cells of layer k) and xy shear (layer k), then the xz/yz
    // shear planes at z = k+1; entries whose results no residual reads (first or
    // last row and column) compute them all the same
    const T cxy = k < nz ? c25 : T(0);
    bool wz = false;
    const bool az = edge_ok(k + 1, nz, g.clamp[4], g.clamp[5], wz);
    const T cz = az ? c25 : T(0);
    const T s1 = wz ? T(2) : T(1);
    const T* U0 = &sm.u[cur][0][0][0];
    const T* U1 = &sm.u[cur][1][0][0];
    const T* U2 = &sm.u[cur][2][0][0];
    const T* U0u = &sm.u[up][0][0][0];
    const T* U1u = &sm.u[up][1][0][0];
    const T* U2u = &sm.u[up][2][0][0];
    const T* EC = &sm.e[cur][0][0];
    const T* EU = &sm.e[up][0][0];
#pragma unroll
    for (int e = 0; e < NE; ++e) {
      if (!wave_has_entry<TY>(e)) continue;
      const int q = en[e].q;
      // every LDS operand of the entry is read before any is used, so that the
      // reads are in flight together (the scheduling barrier keeps the compiler
      // from interleaving each read with its use)
      const T ev = EC[q], e_w = EC[q - 1], e_s = EC[q - LX], e_sw = EC[q - LX - 1];
      const T eu = EU[q], eu_w = EU[q - 1], eu_s = EU[q - LX];
      const T u0 = U0[q], u0e = U0[q + 1], u0s = U0[q - LX];
      const T u1 = U1[q], u1n = U1[q + LX], u1w = U1[q - 1];
      const T u2 = U2[q], u2u = U2u[q], u2uw = U2u[q - 1], u2us = U2u[q - LX];
      const T u0u = U0u[q], u1u = U1u[q];
      __builtin_amdgcn_sched_barrier(0);
      const T exx = (u0e - u0) * rh;
      const T eyy = (u1n - u1) * rh;
      const T ezz = (u2u - u2) * rh;
      T sxx, syy, szz;
      el3d::normal_stress<T>(ev * lam0, T(2) * (ev * mu0), exx, eyy, ezz, sxx, syy, szz);
      const T m = (cxy * (((e_sw + e_s) + e_w) + ev)) * en[e].fxy;
      const T gam = el3d::shear_strain<T>(u0, u0s, u1, u1w, rh);
      // xz edge (i, j+1/2, k+1): cells (i-1..i, j, k..k+1); yz edge (i+1/2, j, k+1)
      const T fxz = fmin(en[e].fxz * s1, T(2));
      const T fyz = fmin(en[e].fyz * s1, T(2));
      const T mxz = (cz * (((e_w + ev) + eu_w) + eu)) * fxz;
      const T gxz = el3d::shear_strain<T>(u0u, u0, u2u, u2uw, rh);
      const T myz = (cz * (((e_s + ev) + eu_s) + eu)) * fyz;
      const T gyz = el3d::shear_strain<T>(u1u, u1, u2u, u2us, rh);
      (&sm.sxx[0][0])[q] = sxx;
      (&sm.syy[0][0])[q] = syy;
      (&sm.szz[0][0])[q] = szz;
      (&sm.txy[0][0])[q] = m * gam;
      (&sm.txz[up][0][0])[q] = mxz * gxz;
      (&sm.tyz[up][0][0])[q] = myz * gyz;
    }
    __syncthreads();
    // residuals and update of the own position at layer k (reads stress planes only)
    const T* SXX = &sm.sxx[0][0];
    const T* SYY = &sm.syy[0][0];
    const T* TXY = &sm.txy[0][0];
    const T* TXZc = &sm.txz[cur][0][0];
    const T* TXZu = &sm.txz[up][0][0];
    const T* TYZc = &sm.tyz[cur][0][0];
    const T* TYZu = &sm.tyz[up][0][0];
    const T szz_cur = (&sm.szz[0][0])[qo];
    T rr[3];
    rr[0] = el3d::residual<T>(bv[0], h2, SXX[qo], SXX[qo - 1], TXY[qo + LX], TXY[qo], TXZu[qo], TXZc[qo]);
    rr[1] = el3d::residual<T>(bv[1], h2, SYY[qo], SYY[qo - LX], TXY[qo + 1], TXY[qo], TYZu[qo], TYZc[qo]);
    rr[2] = el3d::residual<T>(bv[2], h2, szz_cur, szz_prev, TXZc[qo + 1], TXZc[qo], TYZc[qo + LX], TYZc[qo]);
    Out<T, MODE> o[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      o[c].v = MODE == kRefine ? nullptr : A.v + c * pl + kS;
      o[c].u = MODE == kSweep || MODE == kCheck ? A.uout + c * pl + kS : nullptr;
      o[c].r32 = MODE == kRefine ? A.b32 + c * pl + kS : nullptr;
    }
    const bool fixz = (k == 0 && g.fixn[4]) || (k == nz && g.fixn[5]);
    if (plain && k < nz && !fixz) {
      // every lane of the wave owns three free unknowns
#pragma unroll
      for (int c = 0; c < 3; ++c) finish<T, MODE>(o[c], po, false, rr[c], uo[c], vv[c], ca, cc, dt, acc);
    } else {
      unsigned ow = own;
      asm volatile("" : "+v"(ow));   // re-derive the lane tests here, not across the loop
      if (ow & kIn) {
        const unsigned okm = k < nz ? (kOkx | kOky | kOkz) : kOkz;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          if ((ow & okm & (kOkx << c)) == 0u) {
            zero_slot<T, MODE>(o[c], po);
            continue;
          }
          bool fixc = c == 0 ? (ow & kFixx) != 0u : (c == 1 ? (ow & kFixy) != 0u : fixz);
          if (g.pins != nullptr) fixc = fixc || pinned3s(g.pins, c * pl + kS + po / W);
          finish<T, MODE>(o[c], po, fixc, rr[c], uo[c], vv[c], ca, cc, dt, acc);
        }
      }
    }
    if (edge_duty) {
      unsigned ow = own;
      asm volatile("" : "+v"(ow));
      // the face column i = nx: u_x only (u_y, u_z slots are padding)
      if (ow & kXface) {
        const int eb = 1 + (int)threadIdx.x;
        if (k < nz && (ow & kXfok) != 0u) {
          const T r = el3d::residual<T>(bxe, h2, sm.sxx[eb][XA], sm.sxx[eb][XA - 1], sm.txy[eb + 1][XA],
                                        sm.txy[eb][XA], sm.txz[up][eb][XA], sm.txz[cur][eb][XA]);
          finish<T, MODE>(o[0], peo, g.fixn[1] || pinned3s(g.pins, kS + peo / W), r, uxe, vxe, ca, cc, dt, acc);
        } else {
          zero_slot<T, MODE>(o[0], peo);
        }
        zero_slot<T, MODE>(o[1], peo);
        zero_slot<T, MODE>(o[2], peo);
      }
      // the face row j = ny: u_y only (u_x, u_z slots are padding)
      if (ow & kYface) {
        const int fb = TY + 1;
        if (k < nz && (ow & kYfok) != 0u) {
          const T r = el3d::residual<T>(bye, h2, sm.syy[fb][a], sm.syy[fb - 1][a], sm.txy[fb][a + 1],
                                        sm.txy[fb][a], sm.tyz[up][fb][a], sm.tyz[cur][fb][a]);
          finish<T, MODE>(o[1], pfo, g.fixn[3] || pinned3s(g.pins, pl + kS + pfo / W), r, uye, vye, ca, cc, dt,
                          acc);
        } else {
          zero_slot<T, MODE>(o[1], pfo);
        }
        zero_slot<T, MODE>(o[0], pfo);
        zero_slot<T, MODE>(o[2], pfo);
      }
    }
    szz_prev = szz_cur;
    // the next store writes the plane read before the barrier above, and the
    // stress planes read here are rewritten only after the next barrier
  };
  // the top layer k = nz holds only u_z (its u_x, u_y slots are padding).  Its
  // residual needs sigma_zz of the cell below (szz_prev, the cell above is
  // outside) and the xz / yz shear at z = nz, which the layer below formed
  // before its second barrier, and the state plane nz, staged by that layer: no
  // staging, stress pass or barrier of its own, so the last z-tile takes no
  // longer than the others.
  auto top = [&](auto parity) {
    constexpr int cur = decltype(parity)::value;
    const long kS = (long)nz * S;
    T vz = T(0);
    if (MODE == kSweep || MODE == kCheck) vz = ldo(A.v + kS + 2 * pl, po);
    const T bz = ldo(A.b + kS + 2 * pl, po);
    const T* TXZc = &sm.txz[cur][0][0];
    const T* TYZc = &sm.tyz[cur][0][0];
    const T uz = (&sm.u[cur][2][0][0])[qo];
    const T rz = el3d::residual<T>(bz, h2, T(0), szz_prev, TXZc[qo + 1], TXZc[qo], TYZc[qo + LX], TYZc[qo]);
    Out<T, MODE> o[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      o[c].v = MODE == kRefine ? nullptr : A.v + c * pl + kS;
      o[c].u = MODE == kSweep || MODE == kCheck ? A.uout + c * pl + kS : nullptr;
      o[c].r32 = MODE == kRefine ? A.b32 + c * pl + kS : nullptr;
    }
    unsigned ow = own;
    asm volatile("" : "+v"(ow));
    if (ow & kIn) {
      zero_slot<T, MODE>(o[0], po);
      zero_slot<T, MODE>(o[1], po);
      if (ow & kOkz) {
        bool fixc = g.fixn[5] != 0;
        if (g.pins != nullptr) fixc = fixc || pinned3s(g.pins, 2 * pl + kS + po / W);
        finish<T, MODE>(o[2], po, fixc, rz, uz, vz, ca, cc, dt, acc);
      } else {
        zero_slot<T, MODE>(o[2], po);
      }
    }
    // face column and face row slots of the top layer are padding
    if (edge_duty) {
      if (ow & kXface) {
#pragma unroll
        for (int c = 0; c < 3; ++c) zero_slot<T, MODE>(o[c], peo);
      }
      if (ow & kYface) {
#pragma unroll
        for (int c = 0; c < 3; ++c) zero_slot<T, MODE>(o[c], pfo);
      }
    }
  };
  // Every layer but the last fetches plane k+2, unconditionally: the wait for
  // the own velocity and right-hand side (loaded before the fetch) then leaves
  // the fetch in flight; behind a branch it would have to wait for it too.
  using P0 = std::integral_constant<int, 0>;
  using P1 = std::integral_constant<int, 1>;
  using F1 = std::true_type;
  using F0 = std::false_type;
  int k = k0;
  for (; k + 2 < kend; k += 2) {
    layer(P0(), F1(), k);
    layer(P1(), F1(), k + 1);
  }
  if (kend - k == 2) {
    layer(P0(), F1(), k);
    layer(P1(), F0(), k + 1);
  } else {
    layer(P0(), F0(), k);
  }
  if (top_tile) {
    // the buffer parity of layer nz follows that of the last layer run
    if (((nz - k0) & 1) == 0) top(std::integral_constant<int, 0>());
    else top(std::integral_constant<int, 1>());
  }
  if (MODE == kCheck || MODE == kRefine) {
    const double s = block_sum(acc, sm.red);
    if (threadIdx.x == 0) A.partial[tile] = s;
  }
}

// Three tilings per precision: columns of 64 x TY positions streamed through KZ
// layers.  The large one moves the fewest halo bytes (in FP32 its 16 layers put
// a 256x128x128 grid in one round of two resident workgroups per compute unit,
// with one prologue per column); the smaller ones give small grids enough
// workgroups to fill the chip (the shortest columns trade more z-halo planes,
// mostly L2 hits, for twice the workgroups).
template <typename T, int V> struct Cfg3;
template <> struct Cfg3<float, 1> { static constexpr int TY = 8, KZ = 16; };
template <> struct Cfg3<float, 2> { static constexpr int TY = 4, KZ = 4; };
template <> struct Cfg3<float, 3> { static constexpr int TY = 4, KZ = 2; };
template <> struct Cfg3<double, 1> { static constexpr int TY = 4, KZ = 8; };
template <> struct Cfg3<double, 2> { static constexpr int TY = 4, KZ = 4; };
template <> struct Cfg3<double, 3> { static constexpr int TY = 4, KZ = 2; };

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
  if (fp64) return g.tile3d == 3 ? count_s<double, 3>(g) : g.tile3d == 2 ? count_s<double, 2>(g) : count_s<double, 1>(g);
  return g.tile3d == 3 ? count_s<float, 3>(g) : g.tile3d == 2 ? count_s<float, 2>(g) : count_s<float, 1>(g);
}

int el3d_tiles(const ElGeom& g) {
  const int c[6] = {count_s<float, 1>(g),  count_s<float, 2>(g),  count_s<float, 3>(g),
                    count_s<double, 1>(g), count_s<double, 2>(g), count_s<double, 3>(g)};
  int m = 0;
  for (int x : c) m = x > m ? x : m;
  return m;
}

// The large tiling when it gives two resident workgroups per compute unit;
// otherwise, of the two 64 x 4 column tilings, the one with the smaller modelled
// time: rounds of resident workgroups (four of 256 threads per unit in FP32, two
// in FP64, bounded by registers) times the planes a workgroup stages (its layers
// plus two for the prologue).  Ties go to the longer columns (fewer halo bytes).
int el3d_choose_tiling(const ElGeom& g, bool fp64, int ncu) {
  const int large = fp64 ? count_s<double, 1>(g) : count_s<float, 1>(g);
  if (large >= 2 * ncu) return 1;
  const long slots = (long)(fp64 ? 2 : 4) * ncu;
  auto cost = [&](int count, int kz) { return ((count + slots - 1) / slots) * (kz + 2); };
  const long c2 = fp64 ? cost(count_s<double, 2>(g), Cfg3<double, 2>::KZ) : cost(count_s<float, 2>(g), Cfg3<float, 2>::KZ);
  const long c3 = fp64 ? cost(count_s<double, 3>(g), Cfg3<double, 3>::KZ) : cost(count_s<float, 3>(g), Cfg3<float, 3>::KZ);
  return c3 < c2 ? 3 : 2;
}

template <typename T, int MODE>
int launch_el3d(const ElGeom& g, const ElSweep<T>& a, hipStream_t s) {
  if (g.tile3d == 3) return launch_v<T, 3, MODE>(g, a, s);
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
