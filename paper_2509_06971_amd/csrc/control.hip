// Solve control on the device: material preparation (modulus per cell and the
// largest modulus, which sets the pseudo-time step), per-design setup, the
// check-sweep finalisation (residual norm, stop rule, divergence), and small
// elementwise helpers.  Everything that decides when to stop runs in double and
// in a fixed summation order, so repeated runs are bit-identical.
#include "kernels.hpp"
#include "material.hpp"

namespace petto {
namespace {

struct PhaseModuli {
  double e[kMaxPhase + 1];  // solid phases, then the void
};

template <typename T>
__global__ __launch_bounds__(kBlock) void material_kernel(const T* __restrict__ phi, T* __restrict__ E,
                                                          double* __restrict__ E64, const CellRange* ranges,
                                                          int nphase, long phase_stride, double e0,
                                                          double emin, double p, PhaseModuli pm,
                                                          double* partial_max, int bpd) {
  __shared__ double red[kBlock / kWave];
  const int d = blockIdx.y;
  const CellRange R = ranges[d];
  const double* ep = pm.e;
  double mx = 0.0;
  for (long c = (long)blockIdx.x * kBlock + threadIdx.x; c < R.n; c += (long)gridDim.x * kBlock) {
    double dE[kMaxPhase];
    const double e = modulus<T>(phi, R.off + c, phase_stride, nphase, e0, emin, p, ep, dE);
    E[R.off + c] = (T)e;
    if (E64 != nullptr) E64[R.off + c] = e;
    mx = fmax(mx, e);
  }
  const double m = block_max(mx, red);
  if (threadIdx.x == 0) partial_max[(long)d * bpd + blockIdx.x] = m;
}

__global__ void setup_kernel(SetupArgs A) {
  const int d = blockIdx.x;
  const int lane = threadIdx.x;
  double mx = 0.0;
  for (int b = lane; b < A.blocks_per_design; b += kWave) mx = fmax(mx, A.partial_max[(long)d * A.blocks_per_design + b]);
  mx = wave_max(mx);
  if (lane == 0) {
    SolveState& s = A.st[d];
    const double h = A.h[d];
    const double mmax = mx * A.m0;
    double dt = A.dt_user;
    s.dt_scale = h / sqrt(2.0 * A.ndim * mmax);
    if (!(dt > 0.0)) {
      dt = A.theta > 0.0 ? s.dt_scale * sqrt(A.theta) : h * h / (2.0 * A.ndim * mmax);
    }
    s.theta_min = A.theta;
    s.adapt = A.adapt;
    double hd = h * h;
    if (A.ndim == 3) hd *= h;
    s.dt = dt;
    s.theta = A.theta;
    s.hd = hd;
    s.a = A.theta / (A.theta + dt);
    s.c = dt / ((A.theta + dt) * hd);
    s.fnorm = A.fnorm[d];
    s.tol = A.tol;
    s.rho = INFINITY;
    s.rho_first = INFINITY;
    s.r_pde = INFINITY;
    s.sumsq = 0.0;
    s.iters = 0;
    s.done = 0;
    s.status = 0;
    s.checks = 0;
    s.max_iter = A.max_iter;
    s.check_every = A.check_every;
    s.replay = A.replay;
    s.first_seen = 0;
  }
  if (d == 0 && lane == 0) {
    A.ctl[0] = 0;
    A.ctl[1] = 0;
  }
}

// The three Rayleigh-quotient sums of design d, over the whole wave in a fixed
// order (every lane returns the totals).
__device__ __forceinline__ void rq_sums(const double* prq, int rq_blocks, int d, int lane, double& uu,
                                        double& uf, double& ur) {
  const double* q = prq + (long)d * rq_blocks * 3;
  uu = uf = ur = 0.0;
#pragma unroll 4
  for (int b = lane; b < rq_blocks; b += kWave) {
    uu += q[3 * b];
    uf += q[3 * b + 1];
    ur += q[3 * b + 2];
  }
  uu = wave_sum(uu);
  uf = wave_sum(uf);
  ur = wave_sum(ur);
}

// Critical damping of the mode of the state the sums describe: lam = u.Ku /
// (h^d u.u) with u.Ku = u.F - u.r, theta = 1 / (4 lam) (never below the floor),
// and the step for that theta.  A state without a positive quotient (u = 0)
// leaves the damping as it is.
__device__ __forceinline__ void adapt_damping(SolveState& s, double uu, double uf, double ur) {
  const double uku = uf - ur;
  if (uu > 0.0 && uku > 0.0) {
    const double lam = uku / (s.hd * uu);
    const double th = fmin(fmax(s.theta_min, 0.25 / lam), 1e6);
    const double dt = s.dt_scale * sqrt(th);
    s.theta = th;
    s.dt = dt;
    s.a = th / (th + dt);
    s.c = dt / ((th + dt) * s.hd);
  }
}

// Damping chosen from the starting state of a solve, before its first sweep (a
// warm start then begins at the damping of its own mode rather than at the floor).
__global__ __launch_bounds__(kBlock) void adapt_kernel(SolveState* st, const double* prq, int rq_blocks, int ndes) {
  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
  for (int d = w; d < ndes; d += kBlock / kWave) {
    SolveState& s = st[d];
    if (s.done || !s.adapt) continue;
    double uu, uf, ur;
    rq_sums(prq, rq_blocks, d, lane, uu, uf, ur);
    if (lane == 0) adapt_damping(s, uu, uf, ur);
  }
}

__global__ __launch_bounds__(kBlock) void finalize_kernel(FinalizeArgs A) {
  __shared__ int sh_flags[3];
  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
  for (int d = w; d < A.ndes; d += kBlock / kWave) {
    SolveState& s = A.st[d];
    if (s.done) continue;
    const int t0 = A.tile0 ? A.tile0[d] : 0;
    const int t1 = A.tile0 ? A.tile0[d + 1] : A.ntile;
    double acc = 0.0;
    // (unrolled so that the loads overlap; the additions keep their order)
#pragma unroll 8
    for (int t = t0 + lane; t < t1; t += kWave) acc += A.partial[t];
    acc = wave_sum(acc);
    // the Rayleigh-quotient sums of adaptive damping, over the whole wave in a
    // fixed order (used below only when the design goes on)
    double uu = 0.0, uf = 0.0, ur = 0.0;
    const bool rq = s.adapt && A.prq != nullptr;
    if (rq) rq_sums(A.prq, A.rq_blocks, d, lane, uu, uf, ur);
    if (lane == 0) {
      const double rho = sqrt(acc) / s.fnorm;
      s.sumsq = acc;
      s.rho = rho;
      s.r_pde = sqrt(acc) / s.hd / (double)A.ncell[d];
      s.checks += 1;
      // mode 0 checks the state the block's last sweep started from, after the
      // block ran; mode 1 checks the state itself before the block's sweeps.
      if (A.mode == 0) s.iters += s.check_every;
      if (!s.first_seen) {
        s.first_seen = 1;
        s.rho_first = rho;
      }
      if (!isfinite(rho) || rho > A.div_factor * fmax(s.rho_first, s.tol)) {
        s.status = -3;
        s.done = 1;
      } else if (!s.replay && rho <= s.tol) {
        s.status = 0;
        s.done = 1;
      } else if (s.iters >= s.max_iter) {
        s.status = s.replay ? 0 : 1;
        s.done = 1;
      } else if (A.mode == 1) {
        s.iters += s.check_every;   // the sweeps of this block will run
      }
      // critical damping of the mode of the state at this block boundary
      if (!s.done && rq) adapt_damping(s, uu, uf, ur);
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int all = 1, div = 0, nc = 0;
    for (int d = 0; d < A.ndes; ++d) {
      const SolveState& s = A.st[d];
      all &= (s.done != 0);
      div |= (s.status == -3);
      nc |= (s.status == 1);
    }
    const int seq = A.ctl[0];
    A.ctl[1] = all;
    A.ctl[0] = seq + 1;
    PollRecord* slot = &A.ring[seq % kRing];
    slot->all_done = all;
    slot->any_diverged = div;
    slot->any_not_converged = nc;
    slot->seq = seq;
    __threadfence_system();
  }
  (void)sh_flags;
}

__global__ __launch_bounds__(kBlock) void dot_finalize_kernel(const double* pfu, const double* pen,
                                                              const int* tile0, int ntile, int ndes,
                                                              double* out) {
  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
  for (int d = w; d < ndes; d += kBlock / kWave) {
    const int t0 = tile0 ? tile0[d] : 0;
    const int t1 = tile0 ? tile0[d + 1] : ntile;
    double a = 0.0, b = 0.0;
#pragma unroll 8
    for (int t = t0 + lane; t < t1; t += kWave) {
      a += pfu[t];
      b += pen[t];
    }
    a = wave_sum(a);
    b = wave_sum(b);
    if (lane == 0) {
      out[2 * d] = a;
      out[2 * d + 1] = b;
    }
  }
}

template <typename T>
__global__ void fill_kernel(T* p, long n, T value) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) p[i] = value;
}

__global__ void fold_kernel(double* u, float* d, long n, const int* all_done) {
  if (*all_done) return;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    u[i] += (double)d[i];
    d[i] = 0.f;
  }
}

template <typename U, typename R>
__global__ __launch_bounds__(kBlock) void rq_kernel(const U* __restrict__ u, const R* __restrict__ r,
                                                    const double* __restrict__ F, const StateRange* ranges,
                                                    double* prq) {
  __shared__ double red[kBlock / kWave];
  const int d = blockIdx.y;
  const StateRange R0 = ranges[d];
  double uu = 0.0, uf = 0.0, ur = 0.0;
  for (long q = (long)blockIdx.x * kBlock + threadIdx.x; q < R0.n; q += (long)gridDim.x * kBlock) {
    const double x = (double)u[R0.off + q];
    uu += x * x;
    uf += x * (F != nullptr ? F[R0.off + q] : R0.fsrc);
    ur += x * (double)r[R0.off + q];
  }
  const double a = block_sum(uu, red);
  const double b = block_sum(uf, red);
  const double c = block_sum(ur, red);
  if (threadIdx.x == 0) {
    double* o = prq + ((long)d * gridDim.x + blockIdx.x) * 3;
    o[0] = a;
    o[1] = b;
    o[2] = c;
  }
}

inline int grid_for(long n) {
  long b = (n + kBlock - 1) / kBlock;
  if (b > 4096) b = 4096;
  if (b < 1) b = 1;
  return (int)b;
}

}  // namespace

template <typename T>
void launch_material(const T* phi, T* E, double* E64, const CellRange* ranges, int ndes, long max_cells,
                     int nphase, long phase_stride, double e0, double emin, double p, const double* ep,
                     double* partial_max, int blocks_per_design, hipStream_t s) {
  (void)max_cells;
  PhaseModuli pm{};
  for (int m = 0; m <= nphase && m <= kMaxPhase; ++m) pm.e[m] = ep[m];
  hipLaunchKernelGGL((material_kernel<T>), dim3(blocks_per_design, ndes), dim3(kBlock), 0, s, phi, E, E64,
                     ranges, nphase, phase_stride, e0, emin, p, pm, partial_max, blocks_per_design);
}

template <typename U, typename R>
void launch_rq(const U* u, const R* r, const double* F, const StateRange* ranges, int ndes, int bpd,
               double* prq, hipStream_t s) {
  hipLaunchKernelGGL((rq_kernel<U, R>), dim3(bpd, ndes), dim3(kBlock), 0, s, u, r, F, ranges, prq);
}
template void launch_rq<float, float>(const float*, const float*, const double*, const StateRange*, int, int,
                                      double*, hipStream_t);
template void launch_rq<double, double>(const double*, const double*, const double*, const StateRange*, int, int,
                                        double*, hipStream_t);
template void launch_rq<double, float>(const double*, const float*, const double*, const StateRange*, int, int,
                                       double*, hipStream_t);

void launch_adapt(SolveState* st, const double* prq, int rq_blocks, int ndes, hipStream_t s) {
  hipLaunchKernelGGL(adapt_kernel, dim3(1), dim3(kBlock), 0, s, st, prq, rq_blocks, ndes);
}

void launch_setup(const SetupArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(setup_kernel, dim3(a.ndes), dim3(kWave), 0, s, a);
}

void launch_finalize(const FinalizeArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(finalize_kernel, dim3(1), dim3(kBlock), 0, s, a);
}

void launch_dot_finalize(const double* pfu, const double* pen, const int* tile0, int ntile, int ndes,
                         double* out, hipStream_t s) {
  hipLaunchKernelGGL(dot_finalize_kernel, dim3(1), dim3(kBlock), 0, s, pfu, pen, tile0, ntile, ndes, out);
}

template <typename T>
void launch_fill(T* p, long n, T value, hipStream_t s) {
  hipLaunchKernelGGL((fill_kernel<T>), dim3(grid_for(n)), dim3(kBlock), 0, s, p, n, value);
}

void launch_fold(double* u, float* d, long n, const int* all_done, hipStream_t s) {
  hipLaunchKernelGGL(fold_kernel, dim3(grid_for(n)), dim3(kBlock), 0, s, u, d, n, all_done);
}

template void launch_material<float>(const float*, float*, double*, const CellRange*, int, long, int, long,
                                     double, double, double, const double*, double*, int, hipStream_t);
template void launch_material<double>(const double*, double*, double*, const CellRange*, int, long, int, long,
                                      double, double, double, const double*, double*, int, hipStream_t);
template void launch_fill<float>(float*, long, float, hipStream_t);
template void launch_fill<double>(double*, long, double, hipStream_t);

}  // namespace petto
