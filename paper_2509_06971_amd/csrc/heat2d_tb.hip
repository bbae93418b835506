// Multi-sweep (temporally blocked) 2D heat kernel for batches of designs.
//
// Each work-list tile is the inner (64-2K) x (32-2K) cell block of one design; the
// workgroup stages the 64 x 32 window around it (temperature, velocity, source,
// conductivity, face conductances, Dirichlet terms), runs K sweeps and writes back
// the inner block.  Same arithmetic as the one-sweep kernel (heat_ops.hpp), so
// results are bit-identical for every K; the HBM traffic per sweep drops about K
// times, which is what matters for batches larger than the last-level cache.
//
// Inside the window a wave owns RPW consecutive rows, one cell per lane and row:
// the temperatures of the left and right neighbours are the adjacent lanes (DPP
// wave shifts), those above and below inside the wave's rows are the thread's own
// registers, and only each wave's first and last rows cross to the neighbouring
// waves, through double-buffered LDS rows (one barrier per sweep).
#include "heat_ops.hpp"
#include "kernels.hpp"

#pragma clang fp contract(off)

namespace petto {
namespace {

constexpr int EX = 64, EY = 32;
constexpr int NT = 512;
constexpr int NW = NT / kWave;            // waves (8)
constexpr int RPW = EY / NW;              // consecutive window rows per wave (4)
static_assert(EX == kWave && RPW * NW == EY, "one lane per window column, whole rows per wave");

// Rows exchanged between waves: slot w + 1 holds wave w's row; slots 0 and NW + 1
// (below and above the window) stay zero, like the zero ring around the window.
template <typename T>
struct HTb {
  T t_last[2][NW + 2][EX];                // temperature of each wave's last row (sweep parity)
  T t_first[2][NW + 2][EX];               // ... and of its first row
  T k_last[NW + 2][EX];                   // conductivity of each wave's last / first row (staging)
  T k_first[NW + 2][EX];
  double red[NW];
};

// Value of the lane one to the left (lane - 1) or right (lane + 1); the lane at
// the wave's edge reads zero (bound control).  A lane shift must run with every
// lane of the wave active (a masked-off source lane reads as zero), so the empty
// asm keeps the compiler from moving it into code that only some lanes execute.
template <int CTRL, typename T>
__device__ __forceinline__ T wave_shift(T x) {
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

// K sweeps on the staged window.  Sweep k updates rows [k+1, EY-k-1) only: the
// rows outside lie beyond the dependency cone of the written rows [K, EY-K)
// (a row lies in one wave, so the skip is wave-uniform), and rows a sweep skips
// are never read by a row it updates.  FAST: every window position is a cell.
template <typename T, int K, bool CHECK, bool FAST>
__device__ __forceinline__ void heat_tb_sweeps(HTb<T>& sm, T (&tt)[RPW], T (&vv)[RPW], const T (&bb)[RPW],
                                               const T (&kl)[RPW], const T (&kr)[RPW], const T (&kd)[RPW],
                                               const T (&ku)[RPW], const T (&dd)[RPW], const bool (&cell)[RPW],
                                               int li, int w, T ca, T cc, T dt, double& acc) {
  const int l0 = w * RPW;
  for (int k = 0; k < K; ++k) {
    const int cur = k & 1;
    const T t_below = sm.t_last[cur][w][li];       // row l0 - 1
    const T t_above = sm.t_first[cur][w + 2][li];  // row l0 + RPW
    // every row's new temperature from the old ones (Jacobi), then the update
    T tn[RPW], vn[RPW];
#pragma unroll
    for (int s = 0; s < RPW; ++s) {
      const int lj = l0 + s;
      const T t_l = from_left(tt[s]);
      const T t_r = from_right(tt[s]);
      tn[s] = tt[s];
      vn[s] = vv[s];
      if (lj < k + 1 || lj >= EY - k - 1) continue;
      const T t_d = s > 0 ? tt[s > 0 ? s - 1 : 0] : t_below;
      const T t_u = s + 1 < RPW ? tt[s + 1 < RPW ? s + 1 : s] : t_above;
      const T rr = heat::residual<T>(bb[s], tt[s], kl[s], t_l, kr[s], t_r, kd[s], t_d, ku[s], t_u, dd[s]);
      T un = tt[s], v2 = vv[s];
      heat::update<T>(ca, cc, dt, rr, un, v2);
      const bool live = FAST || cell[s];
      tn[s] = live ? un : tt[s];
      vn[s] = live ? v2 : vv[s];
      if (CHECK && k == K - 1) {
        const bool inner = li >= K && li < EX - K && lj >= K && lj < EY - K && live;
        acc += inner ? (double)rr * (double)rr : 0.0;
      }
    }
#pragma unroll
    for (int s = 0; s < RPW; ++s) {
      tt[s] = tn[s];
      vv[s] = vn[s];
    }
    sm.t_last[cur ^ 1][w + 1][li] = tt[RPW - 1];
    sm.t_first[cur ^ 1][w + 1][li] = tt[0];
    __syncthreads();
  }
}

template <typename T, int K, bool CHECK>
__global__ __launch_bounds__(NT) void heat2d_tb_kernel(HeatSweep<T> A) {
  // stop flags and coefficients are read up front, and the early exit comes after
  // the window loads are issued, so their latencies overlap
  const int all_done = *A.all_done;
  const int tile = xcd_tile(blockIdx.x, A.ntile);
  const HeatTile tl = A.tiles[tile];
  const SolveState* st = &A.st[tl.design];
  const int done = st->done;
  const T ca = T(st->a), cc = T(st->c), dt = T(st->dt);
  const HeatDesign D = A.des[tl.design];
  __shared__ HTb<T> sm;
  const int ie = tl.i0 - K, je = tl.j0 - K;
  // lane = window column; the wave index is wave-uniform (scalar branches)
  const int li = threadIdx.x % EX, w = __builtin_amdgcn_readfirstlane(threadIdx.x / EX);
  const int l0 = w * RPW;
  const int i = ie + li;
  const uint8_t* dir = A.dir + D.dir_off;

  // the rows below and above the window are zero
  if (w == 0) {
    sm.t_last[0][0][li] = T(0);
    sm.t_last[1][0][li] = T(0);
    sm.k_last[0][li] = T(0);
  }
  if (w == NW - 1) {
    sm.t_first[0][NW + 1][li] = T(0);
    sm.t_first[1][NW + 1][li] = T(0);
    sm.k_first[NW + 1][li] = T(0);
  }
  // Every load of every row is issued before any is used (a position outside
  // the design reads the design's first cell and is zeroed afterwards), so the
  // window costs one memory round trip; loads behind a per-row branch had each
  // waited for the row before.  (The Dirichlet side tables are read only for
  // cells on the design's boundary.)
  T tt[RPW], vv[RPW], bb[RPW], kc[RPW], dd[RPW];
  int nd[RPW];
  bool cell[RPW];
#pragma unroll
  for (int s = 0; s < RPW; ++s) {
    const int j = je + l0 + s;
    cell[s] = i >= 0 && i < D.nx && j >= 0 && j < D.ny;
    const long g = D.off + (cell[s] ? (long)j * D.nx + i : 0L);
    tt[s] = A.uin[g];
    vv[s] = A.v[g];
    bb[s] = A.b != nullptr ? A.b[g] : T(D.fsrc);
    kc[s] = A.k[g];
  }
#pragma unroll
  for (int s = 0; s < RPW; ++s) {
    const int j = je + l0 + s;
    nd[s] = (cell[s] && (i == 0 || j == 0 || i == D.nx - 1 || j == D.ny - 1))
                ? heat::dirichlet_count(dir, D.nx, D.ny, i, j) : 0;
  }
  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int s = 0; s < RPW; ++s) {
    tt[s] = cell[s] ? tt[s] : T(0);
    vv[s] = cell[s] ? vv[s] : T(0);
    bb[s] = cell[s] ? bb[s] : T(0);
    kc[s] = cell[s] ? kc[s] : T(0);
    dd[s] = cell[s] ? T(2 * nd[s]) * kc[s] : T(0);
  }
  sm.t_last[0][w + 1][li] = tt[RPW - 1];
  sm.t_first[0][w + 1][li] = tt[0];
  sm.k_last[w + 1][li] = kc[RPW - 1];
  sm.k_first[w + 1][li] = kc[0];
  if (all_done || done) return;   // uniform over the workgroup, before its first barrier
  __syncthreads();
  T kl[RPW], kr[RPW], kd[RPW], ku[RPW];
  {
    const T k_below = sm.k_last[w][li];
    const T k_above = sm.k_first[w + 2][li];
#pragma unroll
    for (int s = 0; s < RPW; ++s) {
      const int j = je + l0 + s;
      const T k_l = from_left(kc[s]);
      const T k_r = from_right(kc[s]);
      const T k_d = s > 0 ? kc[s > 0 ? s - 1 : 0] : k_below;
      const T k_u = s + 1 < RPW ? kc[s + 1 < RPW ? s + 1 : s] : k_above;
      kl[s] = heat::face<T>(kc[s], k_l, i > 0);
      kr[s] = heat::face<T>(kc[s], k_r, i < D.nx - 1);
      kd[s] = heat::face<T>(kc[s], k_d, j > 0);
      ku[s] = heat::face<T>(kc[s], k_u, j < D.ny - 1);
    }
  }
  // a window inside its design: every position is a cell (no selects)
  const bool inner_window = ie >= 0 && je >= 0 && ie + EX <= D.nx && je + EY <= D.ny;
  double acc = 0.0;
  if (inner_window) heat_tb_sweeps<T, K, CHECK, true>(sm, tt, vv, bb, kl, kr, kd, ku, dd, cell, li, w, ca, cc, dt, acc);
  else heat_tb_sweeps<T, K, CHECK, false>(sm, tt, vv, bb, kl, kr, kd, ku, dd, cell, li, w, ca, cc, dt, acc);
#pragma unroll
  for (int s = 0; s < RPW; ++s) {
    const int lj = l0 + s, j = je + lj;
    if (!cell[s] || li < K || li >= EX - K || lj < K || lj >= EY - K) continue;
    const long g = D.off + (long)j * D.nx + i;
    A.uout[g] = tt[s];
    A.vout[g] = vv[s];
  }
  if (CHECK) {
    const double sum = block_sum(acc, sm.red);
    if (threadIdx.x == 0) A.partial[tile] = sum;
  }
}

}  // namespace

template <typename T, int K, bool CHECK>
void launch_heat2d_tb(const HeatSweep<T>& a, hipStream_t s) {
  hipLaunchKernelGGL((heat2d_tb_kernel<T, K, CHECK>), dim3(a.ntile), dim3(NT), 0, s, a);
}

#define PETTO_HTB(T, K)                                                         \
  template void launch_heat2d_tb<T, K, false>(const HeatSweep<T>&, hipStream_t); \
  template void launch_heat2d_tb<T, K, true>(const HeatSweep<T>&, hipStream_t);
PETTO_HTB(float, 2)
PETTO_HTB(float, 4)
PETTO_HTB(float, 5)
PETTO_HTB(float, 8)
PETTO_HTB(float, 10)
PETTO_HTB(double, 2)
PETTO_HTB(double, 4)
PETTO_HTB(double, 5)
#undef PETTO_HTB

}  // namespace petto
