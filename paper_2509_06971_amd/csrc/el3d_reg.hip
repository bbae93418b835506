// 3D staggered-grid elastic sweep in register columns, streamed along z
// (gfx950, FP32 sweeps).
//
// A workgroup owns a column of 64 x RTY positions and marches through its z-layers
// like the LDS-plane kernel (el3d_stream.hip), but every value lives at its own
// position in registers: a wave holds one row of 64 positions (one per lane),
// the neighbours along x are the adjacent lanes (DPP wave shifts), along z the
// thread's own previous and next layers, and only what crosses between rows goes
// through LDS, in row buffers published one layer ahead.  The state is fetched
// two layers ahead of its staging and the velocity one layer ahead of its use.  Two more waves hold the
// halo rows below and above the column (they form only the stresses the column
// reads from them), and one wave the two halo columns at x = i0 - 1 and i0 + 64
// (one lane per row).  One barrier per layer: a layer forms its stresses and
// publishes them together with the next layer's staged values, waits once, then
// takes the residuals and the damped update (Eqs. 3.6, 3.9, 3.10, 3.12).
//
// Every staged value, stress and residual is formed with the operations,
// operands and order of the LDS-plane kernel, so results are bit-identical to it
// (the FP64 residual-norm sum aside, whose order follows the threads).
#include "el3d_entry.hpp"
#include "el3d_ops.hpp"
#include "kernels.hpp"

#pragma clang fp contract(off)

namespace petto {
namespace {

using el3d::Entry;
using el3d::edge_ok;
using el3d::ldo;
using el3d::sto;

constexpr int RX = 64;           // positions of a row = lanes of a wave
constexpr int CR = 32;           // first lane of the right halo column in the column wave

// DPP wave shifts by one lane (bound control set: the lane at the edge reads zero).
__device__ __forceinline__ float from_left(float x) {     // value of lane - 1
  return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, x), 0x138, 0xf, 0xf, true));
}
__device__ __forceinline__ float from_right(float x) {    // value of lane + 1
  return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, x), 0x130, 0xf, 0xf, true));
}

template <int NS>
struct RegSmem {
  // staged values crossing between rows, for layer k at parity k & 1:
  // u_x(k), u_y(k), u_z(k+1), E(k), E(k+1) of every row slot and lane
  float xr[2][NS][RX], yr[2][NS][RX], zr[2][NS][RX], e0r[2][NS][RX], e1r[2][NS][RX];
  // stresses of layer k at parity k & 1
  float syy[2][NS][RX], txy[2][NS][RX];
  // yz shear at z-level kz at kz mod 3 (read one layer after it is formed)
  float tyz[3][NS][RX];
  // halo columns, staged values for layer k at parity k & 1: the left column's
  // u_y(k), u_z(k+1), E(k), E(k+1), the right column's u_x(k)
  float yL[2][NS], zL[2][NS], e0L[2][NS], e1L[2][NS], xR[2][NS];
  // halo-column stresses: sigma_xx of the left column and xy shear of the right
  // column of layer k (parity), xz shear of the right column at z-level kz (mod 3)
  float sxL[2][NS], txR[2][NS], tzR[3][NS];
  // sigma_xx of each row's last lane (read by the face column x = nx)
  float sx63[2][NS];
  double red[NS + 1];
};

struct Raw {
  float x, y, z, e;   // staged u_x, u_y, u_z and cell modulus of one layer
};

// Loads of z-layer kk at the entry's sources (layers clamped into the arrays; a
// layer outside the grid is settled by the multipliers in stage()).
__device__ __forceinline__ Raw fetch(const ElGeom& g, const float* __restrict__ ux, const float* __restrict__ uy,
                                     const float* __restrict__ uz, const float* __restrict__ E, long S, long SE,
                                     const Entry<float>& en, int kk) {
  const int nz = g.nz;
  const int kxy = kk < 0 ? 0 : (kk >= nz ? nz - 1 : kk);
  const int kzs = kk < 0 ? 0 : (kk > nz ? nz : kk);
  Raw r;
  r.x = ldo(ux + kxy * S, en.ox);
  r.y = ldo(uy + kxy * S, en.oy);
  r.z = ldo(uz + kzs * S, en.oz);
  r.e = ldo(E + kxy * SE, en.oe);
  return r;
}

// The staged values of layer kk: inside [0, nz) the xy multipliers apply; a
// z-ghost layer (kk = -1 or nz) holds u_x, u_y reflected across a clamped z side
// (else zero); u_z lives on layers 0..nz and the modulus on 0..nz-1.
__device__ __forceinline__ Raw stage(const ElGeom& g, const Entry<float>& en, const Raw& p, int kk) {
  const int nz = g.nz;
  Raw r;
  if (kk >= 0 && kk < nz) {
    r.x = en.mx * p.x;
    r.y = en.my * p.y;
    r.z = en.mz * p.z;
    r.e = en.me * p.e;
  } else {
    const float gs = ((kk == -1 && g.clamp[4]) || (kk == nz && g.clamp[5])) ? -1.f : 0.f;
    const float sz = (kk >= 0 && kk <= nz) ? 1.f : 0.f;
    r.x = (gs * en.gx) * p.x;
    r.y = (gs * en.gy) * p.y;
    r.z = (sz * en.mz) * p.z;
    r.e = 0.f;
  }
  return r;
}

// Bits of a row-wave thread's own position (as in the plane kernel).
enum : unsigned {
  kIn = 1u, kOkx = 2u, kOky = 4u, kOkz = 8u, kFixx = 16u, kFixy = 32u,
};

__device__ __forceinline__ bool pinned_r(const uint32_t* pins, long k) {
  return pins != nullptr && ((pins[k >> 5] >> (k & 31)) & 1u);
}

template <int MODE>
__device__ __forceinline__ void finish_r(float* v, float* u, unsigned off, bool fix, float r, float un, float vn,
                                         float ca, float cc, float dt, double& acc) {
  r = fix ? 0.f : r;
  if (!fix) el3d::update<float>(ca, cc, dt, r, un, vn);
  sto(v, off, vn);
  sto(u, off, un);
  if (MODE == kCheck) acc += (double)r * (double)r;
}

__device__ __forceinline__ void zero_r(float* u, unsigned off) { sto(u, off, 0.f); }

// RTY rows per workgroup (RTY + 3 waves: the rows, the halo rows below and above,
// the halo columns), RKZ z-layers per workgroup.
template <int RTY, int RKZ, int MODE>
__global__ __launch_bounds__((RTY + 3) * RX) void el3d_reg_kernel(ElGeom g, ElSweep<float> A, int tiles_x,
                                                                  int tiles_y, int ntiles) {
  constexpr int NS = RTY + 2;    // row slots: halo row below, RTY rows, halo row above
  constexpr int kBot = RTY, kTop = RTY + 1, kCol = RTY + 2;   // wave roles after the rows
  static_assert(NS <= CR, "one lane per row slot in each half of the column wave");
  const int done = A.st->done;
  const float ca = float(A.st->a), cc = float(A.st->c), dt = float(A.st->dt);
  constexpr unsigned W = sizeof(float);
  __shared__ RegSmem<NS> sm;
  const int tile = xcd_tile(blockIdx.x, ntiles);
  const int txy_ = tiles_x * tiles_y;
  const int tz = tile / txy_;
  const int trem = tile - tz * txy_;
  const int tyi = trem / tiles_x, txi = trem - tyi * tiles_x;
  const int i0 = txi * RX, j0 = tyi * RTY, k0 = tz * RKZ;
  const int lane = (int)(threadIdx.x % RX);
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / RX));
  const int nx = g.nx, ny = g.ny, nz = g.nz;
  const long pl = g.plane;
  const long S = (long)g.px * g.py;
  const long SE = (long)nx * ny;
  const float* ux = A.uin;
  const float* uy = A.uin + pl;
  const float* uz = A.uin + 2 * pl;
  const float rh = float(1.0 / g.h), h2 = float(g.h * g.h);
  const float lam0 = float(g.lam0), mu0 = float(g.mu0);
  const float c25 = 0.25f * mu0;
  const bool top_tile = tz == ntiles / txy_ - 1;
  const int kend = top_tile ? nz : k0 + RKZ;

  // the position this lane stages: a row wave's own position, a halo row's, or
  // (column wave) the left column x = i0 - 1 in lanes 0..NS-1 and the right
  // column x = i0 + 64 in lanes CR..CR+NS-1, one row slot per lane
  const bool is_row = wave < RTY;
  const bool is_col = wave == kCol;
  int pi, pj, slot;
  if (is_col) {
    const bool right = lane >= CR;
    slot = right ? lane - CR : lane;
    slot = slot < NS ? slot : 0;
    pi = right ? i0 + RX : i0 - 1;
    pj = j0 - 1 + slot;
  } else {
    slot = is_row ? wave + 1 : (wave == kBot ? 0 : NS - 1);
    pi = i0 + lane;
    pj = j0 - 1 + slot;
  }
  const bool left_lane = is_col && lane < NS;
  const bool right_lane = is_col && lane >= CR && lane < CR + NS;
  Entry<float> en;
  el3d::make_entry_at<float>(g, pi, pj, en);

  // duties beyond the row waves: the face column x = nx (right halo column of a
  // tile ending at x = nx - 1) and the face row y = ny (halo row above a tile
  // ending at y = ny - 1)
  // (the row above the column is a face-column row of this tile only as the
  // corner x = nx, y = ny; otherwise it belongs to the next tile up)
  const bool col_duty = right_lane && i0 + RX == nx &&
                        ((slot >= 1 && slot <= RTY && pj <= ny) || (slot == NS - 1 && pj == ny));
  const bool row_duty = wave == kTop && j0 + RTY == ny && pi <= nx;
  // own position of a row wave
  unsigned own = 0u;
  bool plain = false;
  unsigned po = 0u;
  if (is_row) {
    const int i = pi, j = pj;
    const bool in = i <= nx && j <= ny;
    own |= in ? kIn : 0u;
    own |= (in && j < ny) ? kOkx : 0u;
    own |= (in && i < nx) ? kOky : 0u;
    own |= (in && i < nx && j < ny) ? kOkz : 0u;
    const bool fx = (i == 0 && g.fixn[0]) || (i == nx && g.fixn[1]);
    const bool fy = (j == 0 && g.fixn[2]) || (j == ny && g.fixn[3]);
    own |= fx ? kFixx : 0u;
    own |= fy ? kFixy : 0u;
    plain = __builtin_amdgcn_ballot_w64(!(i < nx && j < ny) || fx || fy) == 0 && g.pins == nullptr;
    po = in ? (unsigned)(j * g.px + i) * W : 0u;
  }
  // in-layer offsets of the duty unknowns (a valid slot for every lane)
  const unsigned pfo = row_duty ? (unsigned)(ny * g.px + pi) * W : 0u;
  const unsigned peo = col_duty ? (unsigned)(pj * g.px + nx) * W : 0u;

  // own velocity and right-hand side of layer kk (the right-hand side only on the
  // layers that can hold a nonzero one); loaded one layer ahead of their use
  auto load_vb = [&](int kk, float (&vv)[3], float (&bv)[3]) {
    const long kS = kk * S;
    const bool bk = kk >= A.bk_lo && kk <= A.bk_hi;
#pragma unroll
    for (int c = 0; c < 3; ++c) vv[c] = bv[c] = 0.f;
    if (is_row) {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        vv[c] = ldo(A.v + c * pl + kS, po);
        if (bk) bv[c] = ldo(A.b + c * pl + kS, po);
      }
    } else if (row_duty) {
      vv[1] = ldo(A.v + pl + kS, pfo);
      if (bk) bv[1] = ldo(A.b + pl + kS, pfo);
    } else if (col_duty) {
      vv[0] = ldo(A.v + kS, peo);
      if (bk) bv[0] = ldo(A.b + kS, peo);
    }
  };

  // ---------------------------------------------------------------- prologue
  // stage layers k0-1 (cur), k0 (nxt), k0+1 (nn); planes k0+2 and k0+3 in flight
  // (the state is only read by this launch, so it can be fetched well ahead)
  Raw cur, nxt, nn, P1, P2;
  {
    const Raw a = fetch(g, ux, uy, uz, A.E, S, SE, en, k0 - 1);
    const Raw b = fetch(g, ux, uy, uz, A.E, S, SE, en, k0);
    const Raw c = fetch(g, ux, uy, uz, A.E, S, SE, en, k0 + 1);
    P1 = fetch(g, ux, uy, uz, A.E, S, SE, en, k0 + 2);
    P2 = fetch(g, ux, uy, uz, A.E, S, SE, en, k0 + 3);
    cur = stage(g, en, a, k0 - 1);
    nxt = stage(g, en, b, k0);
    nn = stage(g, en, c, k0 + 1);
  }
  float vn[3], bn[3];
  load_vb(k0, vn, bn);
  // publish the staged values of layer kk (from layers kk, kk + 1 held in c0, c1)
  auto publish = [&](int kk, const Raw& c0, const Raw& c1) {
    const int p = kk & 1;
    if (is_col) {
      if (left_lane) {
        sm.yL[p][slot] = c0.y;
        sm.zL[p][slot] = c1.z;
        sm.e0L[p][slot] = c0.e;
        sm.e1L[p][slot] = c1.e;
      }
      if (right_lane) sm.xR[p][slot] = c0.x;
    } else {
      sm.xr[p][slot][lane] = c0.x;
      sm.yr[p][slot][lane] = c0.y;
      sm.zr[p][slot][lane] = c1.z;
      sm.e0r[p][slot][lane] = c0.e;
      sm.e1r[p][slot][lane] = c1.e;
    }
  };
  publish(k0 - 1, cur, nxt);
  if (done) return;   // uniform over the workgroup, before its first barrier
  __syncthreads();

  // xz / yz shear at z-level kk + 1 from layers kk (c0) and kk + 1 (c1), for a row
  // wave or a halo row (neighbours in the row buffers of parity kk & 1)
  float txz_prev = 0.f, tyz_prev = 0.f, szz_prev = 0.f;
  auto shears_up = [&](int kk, const Raw& c0, const Raw& c1, float& txz, float& tyz) {
    const int p = kk & 1;
    bool wz = false;
    const bool az = edge_ok(kk + 1, nz, g.clamp[4], g.clamp[5], wz);
    const float cz = az ? c25 : 0.f;
    const float s1 = wz ? 2.f : 1.f;
    const float fxz = fminf(en.fxz * s1, 2.f);
    const float fyz = fminf(en.fyz * s1, 2.f);
    // xz edge (i, j+1/2, kk+1): cells (i-1..i, j, kk..kk+1)
    float e_l = from_left(c0.e), e_lu = from_left(c1.e), z_lu = from_left(c1.z);
    if (lane == 0) {
      e_l = sm.e0L[p][slot];
      e_lu = sm.e1L[p][slot];
      z_lu = sm.zL[p][slot];
    }
    const float m = (cz * (((e_l + c0.e) + e_lu) + c1.e)) * fxz;
    txz = m * el3d::shear_strain<float>(c1.x, c0.x, c1.z, z_lu, rh);
    // yz edge (i+1/2, j, kk+1): cells (i, j-1..j, kk..kk+1)
    const int sd = slot > 0 ? slot - 1 : 0;
    const float e_d = sm.e0r[p][sd][lane], e_du = sm.e1r[p][sd][lane], z_du = sm.zr[p][sd][lane];
    const float m2 = (cz * (((e_d + c0.e) + e_du) + c1.e)) * fyz;
    tyz = m2 * el3d::shear_strain<float>(c1.y, c0.y, c1.z, z_du, rh);
  };
  // normal stresses of the cell at layer kk (row wave or halo row)
  auto normals = [&](int kk, const Raw& c0, const Raw& c1, float& sxx, float& syy, float& szz) {
    const int p = kk & 1;
    float x_r = from_right(c0.x);
    if (lane == RX - 1) x_r = sm.xR[p][slot];
    const float y_u = sm.yr[p][slot + 1 < NS ? slot + 1 : slot][lane];
    const float exx = (x_r - c0.x) * rh;
    const float eyy = (y_u - c0.y) * rh;
    const float ezz = (c1.z - c0.z) * rh;
    el3d::normal_stress<float>(c0.e * lam0, 2.f * (c0.e * mu0), exx, eyy, ezz, sxx, syy, szz);
  };
  // xy shear at layer kk (row wave or halo row)
  auto shear_xy = [&](int kk, const Raw& c0) {
    const int p = kk & 1;
    const float cxy = kk < nz ? c25 : 0.f;
    const int sd = slot > 0 ? slot - 1 : 0;
    float y_l = from_left(c0.y), e_l = from_left(c0.e);
    const float e_d = sm.e0r[p][sd][lane];
    float e_dl = from_left(e_d);
    if (lane == 0) {
      y_l = sm.yL[p][slot];
      e_l = sm.e0L[p][slot];
      e_dl = sm.e0L[p][sd];
    }
    const float x_d = sm.xr[p][sd][lane];
    const float m = (cxy * (((e_dl + e_d) + e_l) + c0.e)) * en.fxy;
    return m * el3d::shear_strain<float>(c0.x, x_d, c0.y, y_l, rh);
  };
  // the halo columns' stresses at layer kk (column wave; the inner neighbours are
  // the rows' first and last lanes in the row buffers)
  auto column_stresses = [&](int kk, const Raw& c0, const Raw& c1, float& sxl, float& txr, float& tzr) {
    const int p = kk & 1;
    const int sd = slot > 0 ? slot - 1 : 0;
    // left column: sigma_xx of cell (i0 - 1, j, kk)
    {
      const float x_r = sm.xr[p][slot][0];
      const float y_u = from_right(c0.y);
      const float exx = (x_r - c0.x) * rh;
      const float eyy = (y_u - c0.y) * rh;
      const float ezz = (c1.z - c0.z) * rh;
      float syy_, szz_;
      el3d::normal_stress<float>(c0.e * lam0, 2.f * (c0.e * mu0), exx, eyy, ezz, sxl, syy_, szz_);
    }
    // right column: xy shear at (i0 + 64, j, kk) and xz shear at z-level kk + 1
    {
      const float cxy = kk < nz ? c25 : 0.f;
      const float x_d = from_left(c0.x);
      const float e_d = from_left(c0.e);
      const float y_l = sm.yr[p][slot][RX - 1];
      const float e_l = sm.e0r[p][slot][RX - 1];
      const float e_dl = sm.e0r[p][sd][RX - 1];
      const float m = (cxy * (((e_dl + e_d) + e_l) + c0.e)) * en.fxy;
      txr = m * el3d::shear_strain<float>(c0.x, x_d, c0.y, y_l, rh);
      bool wz = false;
      const bool az = edge_ok(kk + 1, nz, g.clamp[4], g.clamp[5], wz);
      const float cz = az ? c25 : 0.f;
      const float s1 = wz ? 2.f : 1.f;
      const float fxz = fminf(en.fxz * s1, 2.f);
      const float e_lu = sm.e1r[p][slot][RX - 1];
      const float z_lu = sm.zr[p][slot][RX - 1];
      const float m2 = (cz * (((e_l + c0.e) + e_lu) + c1.e)) * fxz;
      tzr = m2 * el3d::shear_strain<float>(c1.x, c0.x, c1.z, z_lu, rh);
    }
  };

  // z-level k0 shears and sigma_zz of cell k0 - 1 (from layers k0 - 1, k0)
  {
    const int kk = k0 - 1;
    if (is_col) {
      float sxl, txr, tzr;
      column_stresses(kk, cur, nxt, sxl, txr, tzr);
      if (right_lane) sm.tzR[(kk + 1) % 3][slot] = tzr;
      txz_prev = tzr;
    } else if (wave != kBot) {
      float txz, tyz;
      shears_up(kk, cur, nxt, txz, tyz);
      sm.tyz[(kk + 1) % 3][slot][lane] = tyz;
      txz_prev = txz;
      tyz_prev = tyz;
      if (is_row) {
        float sxx, syy, szz;
        normals(kk, cur, nxt, sxx, syy, szz);
        szz_prev = szz;
      }
    }
  }
  // rotate to layer k0 and publish its staged values
  cur = nxt;
  nxt = nn;
  nn = stage(g, en, P1, k0 + 2);
  P1 = P2;
  P2 = fetch(g, ux, uy, uz, A.E, S, SE, en, k0 + 4);
  publish(k0, cur, nxt);
  __syncthreads();

  double acc = 0.0;
  for (int k = k0; k < kend; ++k) {
    const long kS = k * S;
    // this layer's velocity and right-hand side (loaded during the last layer);
    // the next layer's are issued now
    float vv[3], bv[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      vv[c] = vn[c];
      bv[c] = bn[c];
    }
    if (k + 1 < kend) load_vb(k + 1, vn, bn);
    const int p = k & 1;
    const int q3 = (k + 1) % 3;
    // ------------------------------------------------------------ stresses of layer k
    float sxx = 0.f, syy = 0.f, szz = 0.f, txy = 0.f, txz = 0.f, tyz = 0.f;
    if (is_row) {
      normals(k, cur, nxt, sxx, syy, szz);
      txy = shear_xy(k, cur);
      shears_up(k, cur, nxt, txz, tyz);
      sm.syy[p][slot][lane] = syy;
      sm.txy[p][slot][lane] = txy;
      sm.tyz[q3][slot][lane] = tyz;
      if (lane == RX - 1) sm.sx63[p][slot] = sxx;
    } else if (wave == kBot) {
      normals(k, cur, nxt, sxx, syy, szz);
      sm.syy[p][slot][lane] = syy;
    } else if (wave == kTop) {
      txy = shear_xy(k, cur);
      shears_up(k, cur, nxt, txz, tyz);
      sm.txy[p][slot][lane] = txy;
      sm.tyz[q3][slot][lane] = tyz;
    } else {
      float sxl, txr, tzr;
      column_stresses(k, cur, nxt, sxl, txr, tzr);
      if (left_lane) sm.sxL[p][slot] = sxl;
      if (right_lane) {
        sm.txR[p][slot] = txr;
        sm.tzR[q3][slot] = tzr;
      }
      txy = txr;
      txz = tzr;
    }
    publish(k + 1, nxt, nn);
    __syncthreads();
    // ------------------------------------------------------------ residuals and update of layer k
    float* vb = A.v + kS;
    float* ub = A.uout + kS;
    if (is_row) {
      float sxx_l = from_left(sxx);
      float txy_r = from_right(txy);
      float txz_pr = from_right(txz_prev);
      if (lane == 0) sxx_l = sm.sxL[p][slot];
      if (lane == RX - 1) {
        txy_r = sm.txR[p][slot];
        txz_pr = sm.tzR[k % 3][slot];
      }
      const float txy_u = sm.txy[p][slot + 1][lane];
      const float syy_d = sm.syy[p][slot - 1][lane];
      const float tyz_pu = sm.tyz[k % 3][slot + 1][lane];
      float rr[3];
      rr[0] = el3d::residual<float>(bv[0], h2, sxx, sxx_l, txy_u, txy, txz, txz_prev);
      rr[1] = el3d::residual<float>(bv[1], h2, syy, syy_d, txy_r, txy, tyz, tyz_prev);
      rr[2] = el3d::residual<float>(bv[2], h2, szz, szz_prev, txz_pr, txz_prev, tyz_pu, tyz_prev);
      const float uo[3] = {cur.x, cur.y, cur.z};
      const bool fixz = (k == 0 && g.fixn[4]) || (k == nz && g.fixn[5]);
      if (plain && !fixz) {
#pragma unroll
        for (int c = 0; c < 3; ++c) finish_r<MODE>(vb + c * pl, ub + c * pl, po, false, rr[c], uo[c], vv[c], ca, cc, dt, acc);
      } else {
        unsigned ow = own;
        asm volatile("" : "+v"(ow));
        if (ow & kIn) {
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            if ((ow & (kOkx << c)) == 0u) {
              zero_r(ub + c * pl, po);
              continue;
            }
            bool fixc = c == 0 ? (ow & kFixx) != 0u : (c == 1 ? (ow & kFixy) != 0u : fixz);
            if (g.pins != nullptr) fixc = fixc || pinned_r(g.pins, c * pl + kS + po / W);
            finish_r<MODE>(vb + c * pl, ub + c * pl, po, fixc, rr[c], uo[c], vv[c], ca, cc, dt, acc);
          }
        }
      }
      szz_prev = szz;
      txz_prev = txz;
      tyz_prev = tyz;
    } else if (wave == kTop) {
      // the face row y = ny: u_y only (u_x, u_z slots are padding)
      float txy_r = from_right(txy);
      if (lane == RX - 1) txy_r = sm.txR[p][slot];
      if (row_duty) {
        const float syy_d = sm.syy[p][slot - 1][lane];
        const float r = el3d::residual<float>(bv[1], h2, 0.f, syy_d, txy_r, txy, tyz, tyz_prev);
        if (pi < nx) {
          const bool fix = g.fixn[3] || pinned_r(g.pins, pl + kS + pfo / W);
          finish_r<MODE>(vb + pl, ub + pl, pfo, fix, r, cur.y, vv[1], ca, cc, dt, acc);
        } else {
          zero_r(ub + pl, pfo);
        }
        zero_r(ub, pfo);
        zero_r(ub + 2 * pl, pfo);
      }
      tyz_prev = tyz;
      txz_prev = txz;
    } else if (is_col) {
      // the face column x = nx: u_x only (u_y, u_z slots are padding)
      const float txy_u = from_right(txy);
      if (col_duty) {
        const float sxx_d = sm.sx63[p][slot];
        const float r = el3d::residual<float>(bv[0], h2, 0.f, sxx_d, txy_u, txy, txz, txz_prev);
        if (pj < ny) {
          const bool fix = g.fixn[1] || pinned_r(g.pins, kS + peo / W);
          finish_r<MODE>(vb, ub, peo, fix, r, cur.x, vv[0], ca, cc, dt, acc);
        } else {
          zero_r(ub, peo);
        }
        zero_r(ub + pl, peo);
        zero_r(ub + 2 * pl, peo);
      }
      txz_prev = txz;
    }
    // rotate to layer k + 1; plane k + 4 in flight
    cur = nxt;
    nxt = nn;
    nn = stage(g, en, P1, k + 3);
    P1 = P2;
    P2 = fetch(g, ux, uy, uz, A.E, S, SE, en, k + 5);
  }
  // the top layer k = nz holds only u_z (its u_x, u_y slots are padding); its
  // residual needs sigma_zz of the cell below and the xz / yz shear at z = nz,
  // formed by the last layer before its barrier
  if (top_tile) {
    const long kS = (long)nz * S;
    float* vb = A.v + kS;
    float* ub = A.uout + kS;
    if (is_row) {
      float txz_pr = from_right(txz_prev);
      if (lane == RX - 1) txz_pr = sm.tzR[nz % 3][slot];
      const float tyz_pu = sm.tyz[nz % 3][slot + 1][lane];
      unsigned ow = own;
      asm volatile("" : "+v"(ow));
      if (ow & kIn) {
        zero_r(ub, po);
        zero_r(ub + pl, po);
        if (ow & kOkz) {
          const float vz = ldo(vb + 2 * pl, po);
          const float bz = (nz >= A.bk_lo && nz <= A.bk_hi) ? ldo(A.b + kS + 2 * pl, po) : 0.f;
          const float rz = el3d::residual<float>(bz, h2, 0.f, szz_prev, txz_pr, txz_prev, tyz_pu, tyz_prev);
          bool fixc = g.fixn[5] != 0;
          if (g.pins != nullptr) fixc = fixc || pinned_r(g.pins, 2 * pl + kS + po / W);
          finish_r<MODE>(vb + 2 * pl, ub + 2 * pl, po, fixc, rz, cur.z, vz, ca, cc, dt, acc);
        } else {
          zero_r(ub + 2 * pl, po);
        }
      }
    } else if (row_duty) {
      zero_r(ub, pfo);
      zero_r(ub + pl, pfo);
      zero_r(ub + 2 * pl, pfo);
    } else if (col_duty) {
      zero_r(ub, peo);
      zero_r(ub + pl, peo);
      zero_r(ub + 2 * pl, peo);
    }
  }
  if (MODE == kCheck) {
    const double s = block_sum(acc, sm.red);
    if (threadIdx.x == 0) A.partial[tile] = s;
  }
}

// Register-column tilings: 64 x 8 positions through 32 layers (t = 4) or 16
// layers (t = 5).
template <int V> struct CfgR;
template <> struct CfgR<4> { static constexpr int TY = 8, KZ = 32; };
template <> struct CfgR<5> { static constexpr int TY = 8, KZ = 16; };

template <int V>
void reg_tiles(const ElGeom& g, int& tx, int& ty, int& tz) {
  tx = (g.nx + RX - 1) / RX;
  ty = (g.ny + CfgR<V>::TY - 1) / CfgR<V>::TY;
  tz = (g.nz + CfgR<V>::KZ - 1) / CfgR<V>::KZ;
}

template <int V, int MODE>
int launch_reg_v(const ElGeom& g, const ElSweep<float>& a, hipStream_t s) {
  int tx, ty, tz;
  reg_tiles<V>(g, tx, ty, tz);
  const int nt = tx * ty * tz;
  constexpr int TY = CfgR<V>::TY, KZ = CfgR<V>::KZ;
  hipLaunchKernelGGL((el3d_reg_kernel<TY, KZ, MODE>), dim3(nt), dim3((TY + 3) * RX), 0, s, g, a, tx, ty, nt);
  return nt;
}

}  // namespace

int el3d_reg_count(const ElGeom& g, int t) {
  int tx, ty, tz;
  if (t == 4) reg_tiles<4>(g, tx, ty, tz);
  else reg_tiles<5>(g, tx, ty, tz);
  return tx * ty * tz;
}

template <int MODE>
int launch_el3d_reg(const ElGeom& g, const ElSweep<float>& a, hipStream_t s) {
  return g.tile3d == 4 ? launch_reg_v<4, MODE>(g, a, s) : launch_reg_v<5, MODE>(g, a, s);
}

template int launch_el3d_reg<kSweep>(const ElGeom&, const ElSweep<float>&, hipStream_t);
template int launch_el3d_reg<kCheck>(const ElGeom&, const ElSweep<float>&, hipStream_t);

}  // namespace petto
