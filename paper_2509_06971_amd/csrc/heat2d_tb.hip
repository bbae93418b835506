// Multi-sweep (temporally blocked) 2D heat kernel for batches of designs.
//
// Each work-list tile is the inner (64-2K) x (32-2K) cell block of one design; the
// workgroup stages the 64 x 32 window around it (temperature, velocity, source,
// conductivity, face conductances, Dirichlet terms), runs K sweeps with the
// temperature exchanged through a double-buffered LDS plane (one barrier per
// sweep) and writes back the inner block.  Same arithmetic as the one-sweep kernel
// (heat_ops.hpp), so results are bit-identical for every K; the HBM traffic per
// sweep drops about K times, which is what matters for batches larger than the
// last-level cache.
#include "heat_ops.hpp"
#include "kernels.hpp"

#pragma clang fp contract(off)

namespace petto {
namespace {

constexpr int EX = 64, EY = 32;
constexpr int NT = 512;
constexpr int RSTEP = NT / EX;
constexpr int PPT = EY / RSTEP;
constexpr int PX = EX + 2, PY = EY + 2;

template <typename T>
struct HTb {
  T t[2][PY][PX];
  T k[PY][PX];
  double red[NT / kWave];
};

// K sweeps on the staged window.  Sweep k updates rows [k+1, EY-k-1) only: the
// rows outside lie beyond the dependency cone of the written rows [K, EY-K)
// (one row per wave, so the skip is wave-uniform), and rows a sweep skips are
// never read by a row it updates.  FAST: every window position is a cell.
template <typename T, int K, bool CHECK, bool FAST>
__device__ __forceinline__ void heat_tb_sweeps(HTb<T>& sm, T (&tt)[PPT], T (&vv)[PPT], const T (&bb)[PPT],
                                               const T (&kl)[PPT], const T (&kr)[PPT], const T (&kd)[PPT],
                                               const T (&ku)[PPT], const T (&dd)[PPT], const bool (&cell)[PPT],
                                               int li, int lw, int c, T ca, T cc, T dt, double& acc) {
  for (int k = 0; k < K; ++k) {
    const int cur = k & 1;
#pragma unroll
    for (int s = 0; s < PPT; ++s) {
      const int lj = lw + s * RSTEP, r = lj + 1;
      if (lj < k + 1 || lj >= EY - k - 1) continue;
      const T rr = heat::residual<T>(bb[s], tt[s], kl[s], sm.t[cur][r][c - 1], kr[s], sm.t[cur][r][c + 1], kd[s],
                                     sm.t[cur][r - 1][c], ku[s], sm.t[cur][r + 1][c], dd[s]);
      T un = tt[s], vn = vv[s];
      heat::update<T>(ca, cc, dt, rr, un, vn);
      const bool live = FAST || cell[s];
      tt[s] = live ? un : tt[s];
      vv[s] = live ? vn : vv[s];
      if (CHECK && k == K - 1) {
        const bool inner = li >= K && li < EX - K && lj >= K && lj < EY - K && live;
        acc += inner ? (double)rr * (double)rr : 0.0;
      }
      sm.t[cur ^ 1][r][c] = tt[s];
    }
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
  // one window row per wave: the row index is wave-uniform (scalar branches)
  const int li = threadIdx.x % EX, lw = __builtin_amdgcn_readfirstlane(threadIdx.x / EX);
  const int c = li + 1, i = ie + li;
  const uint8_t* dir = A.dir + D.dir_off;

  for (int q = threadIdx.x; q < 2 * PX + 2 * EY; q += NT) {
    int r, cc;
    if (q < 2 * PX) { r = q < PX ? 0 : PY - 1; cc = q % PX; }
    else { const int t = q - 2 * PX; r = 1 + t / 2; cc = (t & 1) ? PX - 1 : 0; }
    sm.t[0][r][cc] = T(0);
    sm.t[1][r][cc] = T(0);
    sm.k[r][cc] = T(0);
  }
  T tt[PPT], vv[PPT], bb[PPT], kc[PPT], dd[PPT];
  bool cell[PPT];
#pragma unroll
  for (int s = 0; s < PPT; ++s) {
    const int lj = lw + s * RSTEP, j = je + lj;
    cell[s] = i >= 0 && i < D.nx && j >= 0 && j < D.ny;
    tt[s] = vv[s] = bb[s] = kc[s] = dd[s] = T(0);
    if (cell[s]) {
      const long g = D.off + (long)j * D.nx + i;
      tt[s] = A.uin[g];
      vv[s] = A.v[g];
      bb[s] = A.b != nullptr ? A.b[g] : T(D.fsrc);
      kc[s] = A.k[g];
      const int nd = (i == 0 || j == 0 || i == D.nx - 1 || j == D.ny - 1) ? heat::dirichlet_count(dir, D.nx, D.ny, i, j) : 0;
      dd[s] = T(2 * nd) * kc[s];
    }
    sm.t[0][lj + 1][c] = tt[s];
    sm.k[lj + 1][c] = kc[s];
  }
  if (all_done || done) return;   // uniform over the workgroup, before its first barrier
  __syncthreads();
  T kl[PPT], kr[PPT], kd[PPT], ku[PPT];
#pragma unroll
  for (int s = 0; s < PPT; ++s) {
    const int lj = lw + s * RSTEP, j = je + lj, r = lj + 1;
    kl[s] = heat::face<T>(kc[s], sm.k[r][c - 1], i > 0);
    kr[s] = heat::face<T>(kc[s], sm.k[r][c + 1], i < D.nx - 1);
    kd[s] = heat::face<T>(kc[s], sm.k[r - 1][c], j > 0);
    ku[s] = heat::face<T>(kc[s], sm.k[r + 1][c], j < D.ny - 1);
  }
  // a window inside its design: every position is a cell (no selects)
  const bool inner_window = ie >= 0 && je >= 0 && ie + EX <= D.nx && je + EY <= D.ny;
  double acc = 0.0;
  if (inner_window) heat_tb_sweeps<T, K, CHECK, true>(sm, tt, vv, bb, kl, kr, kd, ku, dd, cell, li, lw, c, ca, cc, dt, acc);
  else heat_tb_sweeps<T, K, CHECK, false>(sm, tt, vv, bb, kl, kr, kd, ku, dd, cell, li, lw, c, ca, cc, dt, acc);
#pragma unroll
  for (int s = 0; s < PPT; ++s) {
    const int lj = lw + s * RSTEP, j = je + lj;
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
