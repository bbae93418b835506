// 2D cell-centred steady heat conduction for a batch of independent designs of
// uneven size (Eq. 2.2 with the damped relaxation of Eq. 2.6).
//
// All designs' 64 x 8 cell tiles form one work list; one launch runs one sweep of
// every unconverged design.  Per-design coefficients and stop flags live in device
// memory, so converged designs retire without host involvement.  Faces between
// cells carry the arithmetic-mean conductivity; Dirichlet faces (T = 0 sinks) act
// through the reflected ghost; other boundary faces are no-flux.
#include "heat_ops.hpp"
#include "kernels.hpp"
#include "material.hpp"

#pragma clang fp contract(off)

namespace petto {
namespace {

constexpr int TX = 64, TY = 8;
constexpr int LX = TX + 2, LY = TY + 2;
constexpr int RPT = TY / (kBlock / TX);

template <typename T>
struct HSmem {
  T t[LY][LX];
  T k[LY][LX];
  double red[kBlock / kWave];
};

// Stage temperature and conductivity of cells [i0-1, i0+TX] x [j0-1, j0+TY]: a
// slot outside the design reads the design's first cell and is zeroed by a
// select, so every load of a thread is issued before the first is used (one
// memory round trip for the tile).
template <typename T>
__device__ inline void load_heat_tile(const HeatDesign& D, const T* __restrict__ u,
                                      const T* __restrict__ kk, int i0, int j0, T (*st)[LX],
                                      T (*sk)[LX]) {
  constexpr int NS = (LY * LX + kBlock - 1) / kBlock;
  T tv[NS], kv[NS];
  bool in[NS];
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    const int idx0 = (int)threadIdx.x + s * kBlock;
    const int idx = idx0 < LY * LX ? idx0 : LY * LX - 1;
    const int lj = idx / LX, li = idx - lj * LX;
    const int i = i0 - 1 + li, j = j0 - 1 + lj;
    in[s] = i >= 0 && i < D.nx && j >= 0 && j < D.ny;
    const long c = D.off + (in[s] ? (long)j * D.nx + i : 0L);
    tv[s] = u[c];
    kv[s] = kk != nullptr ? kk[c] : T(0);
  }
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    const int idx = (int)threadIdx.x + s * kBlock;
    if (idx >= LY * LX) continue;
    const int lj = idx / LX, li = idx - lj * LX;
    st[lj][li] = in[s] ? tv[s] : T(0);
    if (sk != nullptr) sk[lj][li] = in[s] ? kv[s] : T(0);
  }
}

__device__ __forceinline__ int dirichlet_count(const HeatDesign& D, const uint8_t* dir, int i, int j) {
  return heat::dirichlet_count(dir + D.dir_off, D.nx, D.ny, i, j);
}

template <typename T, int MODE>
__global__ __launch_bounds__(kBlock) void heat2d_kernel(HeatSweep<T> A) {
  if (MODE == kSweep || MODE == kCheck || (MODE == kRefine && A.st != nullptr)) {
    if (*A.all_done) return;
  }
  const int t = xcd_tile(blockIdx.x, A.ntile);
  const HeatTile tl = A.tiles[t];
  const HeatDesign D = A.des[tl.design];
  if (MODE == kSweep || MODE == kCheck || (MODE == kRefine && A.st != nullptr)) {
    if (A.st[tl.design].done) return;
  }
  __shared__ HSmem<T> sm;
  const int tx = threadIdx.x & (TX - 1), ty = threadIdx.x / TX;
  const int i = tl.i0 + tx;
  T vv[RPT], bb[RPT];
#pragma unroll
  for (int r = 0; r < RPT; ++r) {
    const int j = tl.j0 + ty + r * (kBlock / TX);
    const bool ok = i < D.nx && j < D.ny;
    const long c = D.off + (long)j * D.nx + i;
    vv[r] = T(0);
    if ((MODE == kSweep || MODE == kCheck) && ok) vv[r] = A.v[c];
    bb[r] = ok ? (A.b != nullptr ? A.b[c] : T(D.fsrc)) : T(0);
  }
  load_heat_tile<T>(D, A.uin, A.k, tl.i0, tl.j0, sm.t, sm.k);
  __syncthreads();
  T ca = T(0), cc = T(0), dt = T(0);
  if (MODE == kSweep || MODE == kCheck) {
    const SolveState* st = &A.st[tl.design];
    ca = T(st->a);
    cc = T(st->c);
    dt = T(st->dt);
  }
  double acc = 0.0;
  const int li = tx + 1;
#pragma unroll
  for (int r = 0; r < RPT; ++r) {
    const int j = tl.j0 + ty + r * (kBlock / TX);
    if (i >= D.nx || j >= D.ny) continue;
    const int lj = ty + r * (kBlock / TX) + 1;
    const long c = D.off + (long)j * D.nx + i;
    const T tc = sm.t[lj][li], kc = sm.k[lj][li];
    const T kl = heat::face<T>(kc, sm.k[lj][li - 1], i > 0);
    const T kr = heat::face<T>(kc, sm.k[lj][li + 1], i < D.nx - 1);
    const T kd = heat::face<T>(kc, sm.k[lj - 1][li], j > 0);
    const T ku = heat::face<T>(kc, sm.k[lj + 1][li], j < D.ny - 1);
    const int nd = (i == 0 || j == 0 || i == D.nx - 1 || j == D.ny - 1) ? dirichlet_count(D, A.dir, i, j) : 0;
    const T rr = heat::residual<T>(bb[r], tc, kl, sm.t[lj][li - 1], kr, sm.t[lj][li + 1], kd, sm.t[lj - 1][li],
                                   ku, sm.t[lj + 1][li], T(2 * nd) * kc);
    if (MODE == kSweep || MODE == kCheck) {
      T un = tc, vn = vv[r];
      heat::update<T>(ca, cc, dt, rr, un, vn);
      A.v[c] = vn;
      A.uout[c] = un;
    } else if (MODE == kResid) {
      A.v[c] = rr;
    } else {
      A.b32[c] = (float)rr;
    }
    if (MODE == kCheck || MODE == kRefine) acc += (double)rr * (double)rr;
  }
  if (MODE == kCheck || MODE == kRefine) {
    const double s = block_sum(acc, sm.red);
    if (threadIdx.x == 0) A.partial[t] = s;
  }
}

template <typename U>
struct HAdjSmem {
  U t[LY][LX];
  U w[LY][LX];
  double red[kBlock / kWave];
};

template <typename U, typename T>
__global__ __launch_bounds__(kBlock) void heat2d_adjoint_kernel(HeatAdjoint<U, T> A) {
  const int t = xcd_tile(blockIdx.x, A.ntile);
  const HeatTile tl = A.tiles[t];
  const HeatDesign D = A.des[tl.design];
  __shared__ HAdjSmem<U> sm;
  const bool same = A.w == A.u;
  load_heat_tile<U>(D, A.u, nullptr, tl.i0, tl.j0, sm.t, nullptr);
  if (!same) load_heat_tile<U>(D, A.w, nullptr, tl.i0, tl.j0, sm.w, nullptr);
  __syncthreads();
  const int tx = threadIdx.x & (TX - 1), ty = threadIdx.x / TX;
  const int i = tl.i0 + tx, li = tx + 1;
  double fu = 0.0, en = 0.0;
  const double ep_dummy[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int r = 0; r < RPT; ++r) {
    const int j = tl.j0 + ty + r * (kBlock / TX);
    if (i >= D.nx || j >= D.ny) continue;
    const int lj = ty + r * (kBlock / TX) + 1;
    const long c = D.off + (long)j * D.nx + i;
    auto W_ = [&](int a, int b) -> double { return same ? (double)sm.t[b][a] : (double)sm.w[b][a]; };
    const double tu = (double)sm.t[lj][li], tw = W_(li, lj);
    fu += (A.F != nullptr ? A.F[c] : D.fsrc) * tu;
    double Buu = 0.0, Bwu = 0.0;
    const int di[4] = {-1, 1, 0, 0}, dj[4] = {0, 0, -1, 1};
    const bool has[4] = {i > 0, i < D.nx - 1, j > 0, j < D.ny - 1};
#pragma unroll
    for (int f = 0; f < 4; ++f) {
      if (!has[f]) continue;
      const double du = tu - (double)sm.t[lj + dj[f]][li + di[f]];
      const double dw = tw - W_(li + di[f], lj + dj[f]);
      Buu += 0.5 * du * du;
      Bwu += 0.5 * dw * du;
    }
    const int nd = (i == 0 || j == 0 || i == D.nx - 1 || j == D.ny - 1) ? dirichlet_count(D, A.dir, i, j) : 0;
    Buu += 2.0 * nd * tu * tu;
    Bwu += 2.0 * nd * tw * tu;
    double dE[kMaxPhase];
    const double k = modulus<T>(A.phi, c, 0, 1, A.e0, A.emin, A.p, ep_dummy, dE);
    en += k * Buu;
    A.grad[c] = (T)(-dE[0] * Bwu);
  }
  const double s1 = block_sum(fu, sm.red);
  const double s2 = block_sum(en, sm.red);
  if (threadIdx.x == 0) {
    A.partial_fu[t] = s1;
    A.partial_en[t] = s2;
  }
}

}  // namespace

template <typename T, int MODE>
void launch_heat2d(const HeatSweep<T>& a, hipStream_t s) {
  hipLaunchKernelGGL((heat2d_kernel<T, MODE>), dim3(a.ntile), dim3(kBlock), 0, s, a);
}

template <typename U, typename T>
void launch_heat2d_adjoint(const HeatAdjoint<U, T>& a, hipStream_t s) {
  hipLaunchKernelGGL((heat2d_adjoint_kernel<U, T>), dim3(a.ntile), dim3(kBlock), 0, s, a);
}

template void launch_heat2d<float, kSweep>(const HeatSweep<float>&, hipStream_t);
template void launch_heat2d<float, kCheck>(const HeatSweep<float>&, hipStream_t);
template void launch_heat2d<float, kResid>(const HeatSweep<float>&, hipStream_t);
template void launch_heat2d<double, kSweep>(const HeatSweep<double>&, hipStream_t);
template void launch_heat2d<double, kCheck>(const HeatSweep<double>&, hipStream_t);
template void launch_heat2d<double, kResid>(const HeatSweep<double>&, hipStream_t);
template void launch_heat2d<double, kRefine>(const HeatSweep<double>&, hipStream_t);
template void launch_heat2d_adjoint<float, float>(const HeatAdjoint<float, float>&, hipStream_t);
template void launch_heat2d_adjoint<double, float>(const HeatAdjoint<double, float>&, hipStream_t);
template void launch_heat2d_adjoint<double, double>(const HeatAdjoint<double, double>&, hipStream_t);

}  // namespace petto
