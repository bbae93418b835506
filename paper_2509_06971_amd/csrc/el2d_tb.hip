// Multi-sweep (temporally blocked) 2D elastic APT kernel for gfx950.
//
// A workgroup stages an EX x EY window of grid positions (state, velocity,
// right-hand side, moduli) once, runs K sweeps on it with the state held in
// registers, and writes back the inner (EX-2K) x (EY-2K) positions, whose K-step
// dependency cone lies inside the window.  Each sweep: (B) every position forms
// its cell's normal stresses and its vertex's shear stress, (C) every unknown
// takes the stress jumps around it (Eqs. 3.6, 3.9) and the damped update of
// Eq. 3.12.  The arithmetic is the one of the one-sweep kernel (el2d_ops.hpp),
// so results are bit-identical for every K.  Per-sweep global traffic drops by
// about K times.
//
// Data movement inside the window: a wave owns RPW consecutive window rows, one
// position per lane and row.  Neighbours along x are the adjacent lanes (DPP
// wave shifts, no memory); neighbours along y inside the wave's rows are the
// thread's own registers; only each wave's first and last rows cross to the
// neighbouring waves, through small LDS row buffers (two stores and two loads
// per thread and phase).
#include "el2d_ops.hpp"
#include "kernels.hpp"

#pragma clang fp contract(off)

namespace petto {
namespace {

constexpr int EX = 64, EY = 32;          // window of positions
constexpr int NT = 512;                   // threads
constexpr int NW = NT / kWave;            // waves (8)
constexpr int RPW = EY / NW;              // consecutive window rows per wave (4)
static_assert(EX == kWave && RPW * NW == EY, "one lane per window column, whole rows per wave");

// Rows exchanged between waves: slot w + 1 holds wave w's row; slots 0 and NW + 1
// (below the window and above it) stay zero, like the zero ring around the window.
template <typename T>
struct TbSmem {
  T ux_last[NW + 2][EX];                  // u_x of each wave's last row
  T uy_first[NW + 2][EX];                 // u_y of each wave's first row
  T syy_last[NW + 2][EX];                 // sigma_yy of each wave's last row
  T tau_first[NW + 2][EX];                // shear stress of each wave's first row
  T e_last[NW + 2][EX];                   // cell modulus of each wave's last row (staging)
  double red[NW];
};

// Value of the lane one to the left (lane - 1) or right (lane + 1) in the wave;
// the lane at the wave's edge receives zero (the zero ring around the window).
template <int CTRL, typename T>
__device__ __forceinline__ T wave_shift(T x) {
  // bound control set: a lane whose source lies outside the wave receives zero.
  // A lane shift must run with every lane of the wave active (a source lane that
  // is masked off reads as zero), so the empty asm keeps the compiler from moving
  // it into code that only some lanes execute (such as one arm of a per-lane
  // select).
  if constexpr (sizeof(T) == 4) {
    int r = __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, x), CTRL, 0xf, 0xf, true);
    asm volatile("" : "+v"(r));
    return __builtin_bit_cast(T, r);
  } else {
    const unsigned long long b = __builtin_bit_cast(unsigned long long, x);
    int lo = __builtin_amdgcn_mov_dpp((int)(unsigned)b, CTRL, 0xf, 0xf, true);
    int hi = __builtin_amdgcn_mov_dpp((int)(unsigned)(b >> 32), CTRL, 0xf, 0xf, true);
    asm volatile("" : "+v"(lo), "+v"(hi));
    return __builtin_bit_cast(T, ((unsigned long long)(unsigned)hi << 32) | (unsigned long long)(unsigned)lo);
  }
}
template <typename T>
__device__ __forceinline__ T from_left(T x) { return wave_shift<0x138>(x); }   // wave_shr:1
template <typename T>
__device__ __forceinline__ T from_right(T x) { return wave_shift<0x130>(x); }  // wave_shl:1

__device__ __forceinline__ bool pinned_tb(const uint32_t* pins, long k) {
  return pins != nullptr && ((pins[k >> 5] >> (k & 31)) & 1u);
}

// K sweeps on the staged window.  Sweep k only forms the stresses of rows
// [k, EY-k) and updates rows [k+1, EY-k-1): the values outside lie beyond the
// dependency cone of the written inner rows [K, EY-K), so skipping them leaves
// those rows unchanged (a row lies in one wave, so the skip is wave-uniform).
// FAST: the window is inside the grid with no pins (no ghosts, every unknown free).
template <typename T, int K, bool CHECK, bool FAST>
__device__ __forceinline__ void tb_sweeps(const ElGeom& g, TbSmem<T>& sm, T (&ux)[RPW], T (&uy)[RPW], T (&vx)[RPW],
                                          T (&vy)[RPW], const T (&bx)[RPW], const T (&by)[RPW], const T (&lam)[RPW],
                                          const T (&mu2)[RPW], const T (&mue)[RPW], const T (&fx)[RPW],
                                          const T (&fy)[RPW], int i, int li, int w, int je, T ca, T cc, T dt,
                                          double& acc) {
  const int nx = g.nx, ny = g.ny;
  // reflected-ghost multipliers of clamped sides (0 on other sides), applied on the
  // first / last row and column of the grid
  const T gb = g.clamp[2] ? T(-1) : T(0), gt = g.clamp[3] ? T(-1) : T(0);
  const T gl = g.clamp[0] ? T(-1) : T(0), gr = g.clamp[1] ? T(-1) : T(0);
  const int l0 = w * RPW;                 // first window row of this wave
  // rows skipped by a sweep keep their last stresses; none is read for a kept
  // result, and the zero start keeps every lane shift well defined
  T sxx[RPW], syy[RPW], tau[RPW];
#pragma unroll
  for (int s = 0; s < RPW; ++s) sxx[s] = syy[s] = tau[s] = T(0);
  for (int k = 0; k < K; ++k) {
    // (B) stresses of the cell and the vertex at every position of rows [k, EY-k)
    const T ux_prev = sm.ux_last[w][li];          // row l0 - 1
    const T uy_next = sm.uy_first[w + 2][li];     // row l0 + RPW
#pragma unroll
    for (int s = 0; s < RPW; ++s) {
      const int lj = l0 + s, j = je + lj;
      // x neighbours are lane shifts, so every lane of the wave takes part
      const T ux_r = from_right(ux[s]);
      const T uy_lf = from_left(uy[s]);
      if (lj < k || lj >= EY - k) continue;
      const T uxs = ux[s], uys = uy[s];
      const T uy_u = s + 1 < RPW ? uy[s + 1 < RPW ? s + 1 : s] : uy_next;
      const T ux_dn = s > 0 ? ux[s > 0 ? s - 1 : 0] : ux_prev;
      T ux_below = ux_dn, uy_left = uy_lf, ux_here = uxs, uy_here = uys;
      if (!FAST) {
        // reflected ghosts of clamped sides, as the one-sweep kernel stages them
        ux_below = j == 0 ? gb * uxs : ux_dn;
        uy_left = i == 0 ? gl * uys : uy_lf;
        ux_here = j == ny ? gt * ux_dn : uxs;
        uy_here = i == nx ? gr * uy_lf : uys;
      }
      const T exx = ux_r - uxs;
      const T eyy = uy_u - uys;
      el2d::normal_stress<T>(lam[s], mu2[s], exx, eyy, sxx[s], syy[s]);
      tau[s] = mue[s] * el2d::shear_strain<T>(ux_here, ux_below, uy_here, uy_left);
    }
    sm.syy_last[w + 1][li] = syy[RPW - 1];
    sm.tau_first[w + 1][li] = tau[0];
    __syncthreads();
    // (C) residuals and the damped update of every free unknown of rows [k+1, EY-k-1)
    const T syy_prev = sm.syy_last[w][li];
    const T tau_next = sm.tau_first[w + 2][li];
#pragma unroll
    for (int s = 0; s < RPW; ++s) {
      const int lj = l0 + s;
      const T sxx_lf = from_left(sxx[s]);
      const T tau_r = from_right(tau[s]);
      if (lj < k + 1 || lj >= EY - k - 1) continue;
      const T t0 = tau[s];
      const T tau_u = s + 1 < RPW ? tau[s + 1 < RPW ? s + 1 : s] : tau_next;
      const T syy_dn = s > 0 ? syy[s > 0 ? s - 1 : 0] : syy_prev;
      const T rx = el2d::residual<T>(bx[s], sxx[s], sxx_lf, tau_u, t0);
      const T ry = el2d::residual<T>(by[s], syy[s], syy_dn, tau_r, t0);
      T ux2 = ux[s], vx2 = vx[s], uy2 = uy[s], vy2 = vy[s];
      el2d::update<T>(ca, cc, dt, rx, ux2, vx2);
      el2d::update<T>(ca, cc, dt, ry, uy2, vy2);
      const bool frx = FAST || fx[s] != T(0), fry = FAST || fy[s] != T(0);
      ux[s] = frx ? ux2 : ux[s];
      vx[s] = frx ? vx2 : vx[s];
      uy[s] = fry ? uy2 : uy[s];
      vy[s] = fry ? vy2 : vy[s];
      if (CHECK && k == K - 1) {
        const bool inner = li >= K && li < EX - K && lj >= K && lj < EY - K;
        const double rx2 = (inner && frx) ? (double)rx * (double)rx : 0.0;
        const double ry2 = (inner && fry) ? (double)ry * (double)ry : 0.0;
        acc += rx2 + ry2;
      }
    }
    sm.ux_last[w + 1][li] = ux[RPW - 1];
    sm.uy_first[w + 1][li] = uy[0];
    __syncthreads();
  }
}

template <typename T, int K, bool CHECK>
__global__ __launch_bounds__(NT) void el2d_tb_kernel(ElGeom g, ElSweep<T> A, int tiles_x, int ntiles) {
  static_assert(EX - 2 * K > 0 && EY - 2 * K > 0, "window too small for K sweeps");
  // the stop flag and coefficients are read up front, so their latency overlaps
  // the window loads; the early exit comes after the loads are issued
  const int done = A.st->done;
  const T ca = T(A.st->a), cc = T(A.st->c), dt = T(A.st->dt);
  constexpr int TXI = EX - 2 * K, TYI = EY - 2 * K;
  __shared__ TbSmem<T> sm;
  const int tile = xcd_tile(blockIdx.x, ntiles);
  const int tyi = tile / tiles_x, txi = tile - tyi * tiles_x;
  const int ie = txi * TXI - K, je = tyi * TYI - K;     // window origin
  // lane = window column; the wave index is wave-uniform (scalar branches)
  const int li = threadIdx.x % EX, w = __builtin_amdgcn_readfirstlane(threadIdx.x / EX);
  const int l0 = w * RPW;
  const int nx = g.nx, ny = g.ny, px = g.px;
  const long pl = g.plane;
  const int i = ie + li;

  // the rows below and above the window are zero
  if (w == 0) {
    sm.ux_last[0][li] = T(0);
    sm.syy_last[0][li] = T(0);
    sm.e_last[0][li] = T(0);
  }
  if (w == NW - 1) {
    sm.uy_first[NW + 1][li] = T(0);
    sm.tau_first[NW + 1][li] = T(0);
  }

  T ux[RPW], uy[RPW], vx[RPW], vy[RPW], bx[RPW], by[RPW], lam[RPW], mu2[RPW], mue[RPW], e[RPW];
  T fx[RPW], fy[RPW];                       // 1 for a free unknown, 0 otherwise
#pragma unroll
  for (int s = 0; s < RPW; ++s) {
    const int j = je + l0 + s;
    const bool validx = i >= 0 && i <= nx && j >= 0 && j < ny;
    const bool validy = i >= 0 && i < nx && j >= 0 && j <= ny;
    const long p = (long)j * px + i;
    ux[s] = vx[s] = bx[s] = uy[s] = vy[s] = by[s] = T(0);
    fx[s] = fy[s] = T(0);
    if (validx) {
      ux[s] = A.uin[p];
      vx[s] = A.v[p];
      bx[s] = A.b[p];
      const bool fix = (i == 0 && g.fixn[0]) || (i == nx && g.fixn[1]) || pinned_tb(g.pins, p);
      fx[s] = fix ? T(0) : T(1);
    }
    if (validy) {
      uy[s] = A.uin[pl + p];
      vy[s] = A.v[pl + p];
      by[s] = A.b[pl + p];
      const bool fix = (j == 0 && g.fixn[2]) || (j == ny && g.fixn[3]) || pinned_tb(g.pins, pl + p);
      fy[s] = fix ? T(0) : T(1);
    }
    const bool cell = i >= 0 && i < nx && j >= 0 && j < ny;
    e[s] = cell ? A.E[(long)j * nx + i] : T(0);
  }
  sm.e_last[w + 1][li] = e[RPW - 1];
  sm.ux_last[w + 1][li] = ux[RPW - 1];
  sm.uy_first[w + 1][li] = uy[0];
  if (done) return;   // uniform over the workgroup, before its first barrier
  __syncthreads();
  const T lam0 = T(g.lam0), mu0 = T(g.mu0);
  {
    const T e_prev = sm.e_last[w][li];                 // cells of row l0 - 1
#pragma unroll
    for (int s = 0; s < RPW; ++s) {
      const int j = je + l0 + s;
      const T es = e[s];
      const T ed = s > 0 ? e[s > 0 ? s - 1 : 0] : e_prev;   // cell below
      const T e_lf = from_left(es);                          // cell to the left
      const T ed_lf = from_left(ed);                         // cell below-left
      lam[s] = es * lam0;
      mu2[s] = T(2) * (es * mu0);
      bool act = i >= 0 && j >= 0 && i <= nx && j <= ny, on = false;
      if (i == 0) { act = act && g.clamp[0]; on = true; }
      if (i == nx) { act = act && g.clamp[1]; on = true; }
      if (j == 0) { act = act && g.clamp[2]; on = true; }
      if (j == ny) { act = act && g.clamp[3]; on = true; }
      mue[s] = el2d::vertex_modulus<T>(mu0, ed_lf, ed, e_lf, es, act, on);
    }
  }

  // A window that lies strictly inside the grid and holds no pinned unknown has
  // no ghosts and no fixed unknowns: its sweeps skip those selects.
  const bool inner_window = ie >= 1 && je >= 1 && ie + EX <= nx && je + EY <= ny && g.pins == nullptr;
  double acc = 0.0;
  if (inner_window) {
    tb_sweeps<T, K, CHECK, true>(g, sm, ux, uy, vx, vy, bx, by, lam, mu2, mue, fx, fy, i, li, w, je, ca, cc, dt,
                                 acc);
  } else {
    tb_sweeps<T, K, CHECK, false>(g, sm, ux, uy, vx, vy, bx, by, lam, mu2, mue, fx, fy, i, li, w, je, ca, cc, dt,
                                  acc);
  }
  // write back the inner positions (padding slots of the grid get zero)
#pragma unroll
  for (int s = 0; s < RPW; ++s) {
    const int lj = l0 + s, j = je + lj;
    if (li < K || li >= EX - K || lj < K || lj >= EY - K) continue;
    if (i > nx || j > ny) continue;
    const long p = (long)j * px + i;
    A.uout[p] = j < ny ? ux[s] : T(0);
    if (j < ny) A.vout[p] = vx[s];
    A.uout[pl + p] = i < nx ? uy[s] : T(0);
    if (i < nx) A.vout[pl + p] = vy[s];
  }
  if (CHECK) {
    const double sum = block_sum(acc, sm.red);
    if (threadIdx.x == 0) A.partial[tile] = sum;
  }
}

template <int K>
void tb_tiles(const ElGeom& g, int& tx, int& ty) {
  tx = (g.nx + 1 + (EX - 2 * K) - 1) / (EX - 2 * K);
  ty = (g.ny + 1 + (EY - 2 * K) - 1) / (EY - 2 * K);
}

}  // namespace

int el2d_tb_tiles(const ElGeom& g, int K) {
  int tx = 0, ty = 0;
  switch (K) {
    case 2: tb_tiles<2>(g, tx, ty); break;
    case 4: tb_tiles<4>(g, tx, ty); break;
    case 5: tb_tiles<5>(g, tx, ty); break;
    case 8: tb_tiles<8>(g, tx, ty); break;
    case 10: tb_tiles<10>(g, tx, ty); break;
    default: return 0;
  }
  return tx * ty;
}

template <typename T, int K, bool CHECK>
int launch_el2d_tb(const ElGeom& g, const ElSweep<T>& a, hipStream_t s) {
  int tx, ty;
  tb_tiles<K>(g, tx, ty);
  const int nt = tx * ty;
  hipLaunchKernelGGL((el2d_tb_kernel<T, K, CHECK>), dim3(nt), dim3(NT), 0, s, g, a, tx, nt);
  return nt;
}

#define PETTO_TB(T, K)                                                                 \
  template int launch_el2d_tb<T, K, false>(const ElGeom&, const ElSweep<T>&, hipStream_t); \
  template int launch_el2d_tb<T, K, true>(const ElGeom&, const ElSweep<T>&, hipStream_t);
PETTO_TB(float, 2)
PETTO_TB(float, 4)
PETTO_TB(float, 5)
PETTO_TB(float, 8)
PETTO_TB(float, 10)
PETTO_TB(double, 2)
PETTO_TB(double, 4)
PETTO_TB(double, 5)
#undef PETTO_TB

}  // namespace petto
