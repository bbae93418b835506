// Phase-field design update (Sections 2.4 and 3.1).
//
// Default model: normalised sensitivity step (Eq. 3.2 weight alpha_h), one
// explicit Allen-Cahn step with the double-well w = sin^2(pi phi)/64 of Eq. 2.15
// and mirror (no-flux) boundaries, and the volume constraint enforced exactly by a
// uniform shift s: mean(clamp(phi'' + s, 0, ub)) = V.  The shift is found by a
// bracketed 64-way search: each pass evaluates the clamped volume at 63 interior
// candidates of the current bracket in one sweep over the cells (FP64 sums in a
// fixed order) and keeps the sub-interval holding the root.
//
// The paper's own model: the penalty step of Eq. 2.13 and one explicit
// Cahn-Hilliard step of Eq. 2.14 (two mirror-Laplacian passes).
#include "kernels.hpp"

namespace petto {
namespace {

constexpr int kMaxPhaseBlocks = 1024;

template <typename T>
__global__ __launch_bounds__(kBlock) void gmax_kernel(PhaseArgs<T> A) {
  __shared__ double red[kBlock / kWave];
  double m = 0.0;
  for (long c = (long)blockIdx.x * kBlock + threadIdx.x; c < A.n; c += (long)gridDim.x * kBlock)
    m = fmax(m, fabs((double)A.g[c]));
  m = block_max(m, red);
  if (threadIdx.x == 0) A.partial[blockIdx.x] = m;
}

__global__ void gmax_final_kernel(const double* partial, int nb, double* scal) {
  double m = 0.0;
  #pragma unroll 8
  for (int b = threadIdx.x; b < nb; b += kWave) m = fmax(m, partial[b]);
  m = wave_max(m);
  if (threadIdx.x == 0) scal[0] = m;
}

// Bounds of a cell for this phase: design cells [0, 1 - used]; void-region cells
// held at 0; passive-solid cells hold phase 0 at 1 (the later phases then find
// no room, since `used` already counts it).
template <typename T>
__device__ inline void cell_bounds(const PhaseArgs<T>& A, long c, double& lb, double& ub) {
  ub = A.used == nullptr ? 1.0 : 1.0 - A.used[c];
  lb = 0.0;
  if (A.region != nullptr) {
    const uint8_t r = A.region[c];
    if (r == 1) {
      ub = 0.0;
    } else if (r == 2 && A.first) {
      lb = 1.0;
      ub = 1.0;
    }
  }
}

template <typename T>
__device__ inline double sens_step(const PhaseArgs<T>& A, long c, double gmax) {
  const double gh = gmax > 0.0 ? (double)A.g[c] / gmax : 0.0;
  return (double)A.phi[c] - A.alpha * gh;
}

template <typename T>
__global__ __launch_bounds__(kBlock) void step_kernel(PhaseArgs<T> A) {
  __shared__ double red[kBlock / kWave];
  const double gmax = A.scal[0];
  const double rh2 = 1.0 / (A.h * A.h);
  const double kPi = 3.141592653589793;
  double mn = INFINITY, mx = -INFINITY, ubmax = -INFINITY;
  const long sxy = (long)A.nx * A.ny;
  for (long c = (long)blockIdx.x * kBlock + threadIdx.x; c < A.n; c += (long)gridDim.x * kBlock) {
    const int k = (int)(c / sxy);
    const long rem = c - (long)k * sxy;
    const int j = (int)(rem / A.nx), i = (int)(rem - (long)j * A.nx);
    const double x = sens_step(A, c, gmax);
    // mirror boundaries: a missing neighbour takes the cell's own value
    const double xl = i > 0 ? sens_step(A, c - 1, gmax) : x;
    const double xr = i < A.nx - 1 ? sens_step(A, c + 1, gmax) : x;
    const double yl = j > 0 ? sens_step(A, c - A.nx, gmax) : x;
    const double yr = j < A.ny - 1 ? sens_step(A, c + A.nx, gmax) : x;
    double lap = (xl + xr - 2.0 * x) + (yl + yr - 2.0 * x);
    if (A.ndim == 3) {
      const double zl = k > 0 ? sens_step(A, c - sxy, gmax) : x;
      const double zr = k < A.nz - 1 ? sens_step(A, c + sxy, gmax) : x;
      lap += zl + zr - 2.0 * x;
    }
    lap *= rh2;
    const double wp = (kPi / 64.0) * sin(2.0 * kPi * x);
    const double y = x - A.dt_ac * (wp - A.gamma * lap);
    A.work[c] = y;
    mn = fmin(mn, y);
    mx = fmax(mx, y);
    double lb, ub;
    cell_bounds(A, c, lb, ub);
    ubmax = fmax(ubmax, ub);
  }
  const double a = block_min(mn, red);
  const double b = block_max(mx, red);
  const double u = block_max(ubmax, red);
  if (threadIdx.x == 0) {
    A.partial[3 * blockIdx.x] = a;
    A.partial[3 * blockIdx.x + 1] = b;
    A.partial[3 * blockIdx.x + 2] = u;
  }
}

// Initial bracket [-max phi'', max ub - min phi''].
__global__ void bracket_init_kernel(const double* partial, int nb, double* scal, double target) {
  double mn = INFINITY, mx = -INFINITY, ub = -INFINITY;
  #pragma unroll 8
  for (int b = threadIdx.x; b < nb; b += kWave) {
    mn = fmin(mn, partial[3 * b]);
    mx = fmax(mx, partial[3 * b + 1]);
    ub = fmax(ub, partial[3 * b + 2]);
  }
  mn = wave_min(mn);
  mx = wave_max(mx);
  ub = wave_max(ub);
  if (threadIdx.x == 0) {
    scal[1] = -mx;
    scal[2] = ub - mn;
    scal[5] = target;
  }
}

// The candidates go in chunks of kChunk (a thread's sums of one chunk stay in
// registers; the cells are read once per chunk), each sum in the same order as
// with all candidates at once.
constexpr int kChunk = 16;

template <typename T>
__global__ __launch_bounds__(kBlock) void pass_kernel(PhaseArgs<T> A) {
  __shared__ double sh[kBlock / kWave][kCand + 1];
  const double lo = A.scal[1], hi = A.scal[2];
  const double step = (hi - lo) / (kCand + 1);
  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
  for (int k0 = 0; k0 < kCand; k0 += kChunk) {
    double acc[kChunk];
#pragma unroll
    for (int q = 0; q < kChunk; ++q) acc[q] = 0.0;
    for (long c = (long)blockIdx.x * kBlock + threadIdx.x; c < A.n; c += (long)gridDim.x * kBlock) {
      const double x = A.work[c];
      double lb, ub;
      cell_bounds(A, c, lb, ub);
#pragma unroll
      for (int q = 0; q < kChunk; ++q) {
        const int k = k0 + q;
        if (k < kCand) acc[q] += fmin(fmax(x + (lo + (k + 1) * step), lb), ub);
      }
    }
#pragma unroll
    for (int q = 0; q < kChunk; ++q) {
      const double s = wave_sum(acc[q]);
      if (lane == 0 && k0 + q < kCand) sh[w][k0 + q] = s;
    }
  }
  __syncthreads();
  if (threadIdx.x < kCand) {
    double s = 0.0;
    for (int q = 0; q < kBlock / kWave; ++q) s += sh[q][threadIdx.x];
    A.partial[(long)blockIdx.x * (kCand + 1) + threadIdx.x] = s;
  }
}

// Keep the candidate interval holding the root: lo = last candidate with
// V < target, hi = first candidate with V >= target.
__global__ void bracket_kernel(const double* partial, int nb, double* scal) {
  __shared__ double V[kCand];
  const int k = threadIdx.x;
  if (k < kCand) {
    // (unrolled so that many loads are in flight; the additions keep their order)
    double s = 0.0;
#pragma unroll 16
    for (int b = 0; b < nb; ++b) s += partial[(long)b * (kCand + 1) + k];
    V[k] = s;
  }
  __syncthreads();
  if (k == 0) {
    const double lo = scal[1], hi = scal[2], target = scal[5];
    const double step = (hi - lo) / (kCand + 1);
    int first = kCand;
    for (int q = 0; q < kCand; ++q) {
      if (V[q] >= target) { first = q; break; }
    }
    const double nlo = first == 0 ? lo : lo + first * step;
    const double nhi = first == kCand ? hi : lo + (first + 1) * step;
    scal[1] = nlo;
    scal[2] = nhi;
  }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void apply_kernel(PhaseArgs<T> A) {
  __shared__ double red[kBlock / kWave];
  const double s = 0.5 * (A.scal[1] + A.scal[2]);
  double acc = 0.0;
  for (long c = (long)blockIdx.x * kBlock + threadIdx.x; c < A.n; c += (long)gridDim.x * kBlock) {
    double lb, ub;
    cell_bounds(A, c, lb, ub);
    const T y = (T)fmin(fmax(A.work[c] + s, lb), ub);
    A.phi[c] = y;
    acc += (double)y;
    if (A.used_out != nullptr) A.used_out[c] = (A.used == nullptr ? 0.0 : A.used[c]) + (double)y;
  }
  const double t = block_sum(acc, red);
  if (threadIdx.x == 0) A.partial[blockIdx.x] = t;
  if (blockIdx.x == 0 && threadIdx.x == 0) A.scal[3] = s;
}

__global__ void volume_final_kernel(const double* partial, int nb, double* scal, double n) {
  double s = 0.0;
  #pragma unroll 8
  for (int b = threadIdx.x; b < nb; b += kWave) s += partial[b];
  s = wave_sum(s);
  if (threadIdx.x == 0) scal[4] = s / n;
}

// ---- the paper's own update: penalty step (Eq. 2.13, normalised sensitivity of
// Section 3.1) and one explicit Cahn-Hilliard step (Eq. 2.14), every stored
// phase of a design in each launch.  The per-phase block partials and final sums
// keep the cell-to-thread mapping and summation order of a one-phase launch.

// max|g_m|, sum phi_m and (with the void-region term) sum of phi_m over the void
// region; blockIdx.y is the phase
template <typename T>
__global__ __launch_bounds__(kBlock) void pen_reduce_kernel(PenaltyArgs<T> A) {
  __shared__ double red[kBlock / kWave];
  const int m = blockIdx.y;
  const T* g = A.g + (long)m * A.pstride;
  const T* phi = A.phi + (long)m * A.pstride;
  const bool rsum = A.alpha_b != 0.0 && A.region != nullptr;
  double gm = 0.0, s = 0.0, r = 0.0;
  for (long c = (long)blockIdx.x * kBlock + threadIdx.x; c < A.n; c += (long)gridDim.x * kBlock) {
    gm = fmax(gm, fabs((double)g[c]));
    const double f = (double)phi[c];
    s += f;
    if (rsum) r += A.region[c] == 1 ? f : 0.0;
  }
  gm = block_max(gm, red);
  s = block_sum(s, red);
  if (rsum) r = block_sum(r, red);
  if (threadIdx.x == 0) {
    double* q = A.partial + 3 * ((long)m * gridDim.x + blockIdx.x);
    q[0] = gm;
    q[1] = s;
    q[2] = r;
  }
}

// Per phase (one wave each): the three totals and the volume-penalty term
// alpha_v dJ_v/dphi = alpha_v 2 (h^d sum phi - V N h^d) h^d.
template <typename T>
__global__ void pen_final_kernel(PenaltyArgs<T> A) {
  const int m = blockIdx.x;
  const int nb = A.nblocks;
  const double* q = A.partial + 3L * m * nb;
  double gm = 0.0, s = 0.0, r = 0.0;
  #pragma unroll 8
  for (int b = threadIdx.x; b < nb; b += kWave) {
    gm = fmax(gm, q[3 * b]);
    s += q[3 * b + 1];
    r += q[3 * b + 2];
  }
  gm = wave_max(gm);
  s = wave_sum(s);
  r = wave_sum(r);
  if (threadIdx.x == 0) {
    double* sc = A.scal + 8 * m;
    const double hd = A.ndim == 3 ? A.h * A.h * A.h : A.h * A.h;
    const double vpen = A.alpha_v * (2.0 * (hd * s - A.vol_frac[m] * (double)A.n * hd) * hd);
    sc[0] = gm;
    sc[1] = vpen;
    sc[3] = -vpen;
    sc[6] = s;
    sc[7] = r;
  }
}

// phi'_m at cell c: phi - alpha_h g / max|g| - alpha_v dJ_v/dphi - alpha_1 dJ_1/dphi
// - alpha_b dJ_b/dphi, with dJ_1/dphi = 2 (sum_m phi_m - 1) h^d (tot: that sum at c)
// and dJ_b/dphi = 2 h^d (sum over the void region) h^d on the region's cells.
template <typename T>
__device__ inline double pen_value(const PenaltyArgs<T>& A, int m, long c, double tot, double hd) {
  const double* sc = A.scal + 8 * m;
  const double gmax = sc[0];
  const double f = (double)A.phi[(long)m * A.pstride + c];
  const double gh = gmax > 0.0 ? (double)A.g[(long)m * A.pstride + c] / gmax : 0.0;
  double y = (f - A.alpha * gh) - sc[1];
  if (A.alpha_1 != 0.0) y = y - A.alpha_1 * (2.0 * (tot - 1.0) * hd);
  if (A.alpha_b != 0.0 && A.region != nullptr && A.region[c] == 1) y = y - A.alpha_b * (2.0 * (hd * sc[7]) * hd);
  return y;
}

// sum over the stored phases at cell c (only needed by the partition term)
template <typename T>
__device__ inline double phase_total(const PenaltyArgs<T>& A, long c) {
  if (A.alpha_1 == 0.0) return 0.0;
  double t = 0.0;
  for (int m = 0; m < A.nphase; ++m) t += (double)A.phi[(long)m * A.pstride + c];
  return t;
}

// phi'_m of every phase at every cell
template <typename T>
__global__ __launch_bounds__(kBlock) void pen_p1_kernel(PenaltyArgs<T> A) {
  const double hd = A.ndim == 3 ? A.h * A.h * A.h : A.h * A.h;
  for (long c = (long)blockIdx.x * kBlock + threadIdx.x; c < A.n; c += (long)gridDim.x * kBlock) {
    const double tot = phase_total(A, c);
    for (int m = 0; m < A.nphase; ++m) A.p1[(long)m * A.mstride + c] = pen_value(A, m, c, tot, hd);
  }
}

// Mirror-boundary Laplacian of a double field at cell (i, j, k).
__device__ inline double lap_mirror(const double* x, long c, int i, int j, int k, int nx, int ny, int nz, int ndim,
                                    long sxy, double rh2) {
  const double v = x[c];
  const double xl = i > 0 ? x[c - 1] : v;
  const double xr = i < nx - 1 ? x[c + 1] : v;
  const double yl = j > 0 ? x[c - nx] : v;
  const double yr = j < ny - 1 ? x[c + nx] : v;
  double lap = (xl + xr - 2.0 * v) + (yl + yr - 2.0 * v);
  if (ndim == 3) {
    const double zl = k > 0 ? x[c - sxy] : v;
    const double zr = k < nz - 1 ? x[c + sxy] : v;
    lap += zl + zr - 2.0 * v;
  }
  return lap * rh2;
}

// mu_m = w'(phi'_m) - gamma lap(phi'_m), w = sin^2(pi phi) / 64 (Eq. 2.15)
template <typename T>
__global__ __launch_bounds__(kBlock) void pen_mu_kernel(PenaltyArgs<T> A) {
  const double rh2 = 1.0 / (A.h * A.h);
  const double kPi = 3.141592653589793;
  const long sxy = (long)A.nx * A.ny;
  for (long c = (long)blockIdx.x * kBlock + threadIdx.x; c < A.n; c += (long)gridDim.x * kBlock) {
    const int k = (int)(c / sxy);
    const long rem = c - (long)k * sxy;
    const int j = (int)(rem / A.nx), i = (int)(rem - (long)j * A.nx);
    for (int m = 0; m < A.nphase; ++m) {
      const double* x = A.p1 + (long)m * A.mstride;
      const double v = x[c];
      const double wp = (kPi / 64.0) * sin(2.0 * kPi * v);
      A.mu[(long)m * A.mstride + c] = wp - A.gamma * lap_mirror(x, c, i, j, k, A.nx, A.ny, A.nz, A.ndim, sxy, rh2);
    }
  }
}

// phi_m = phi'_m + dt_ch D lap(mu_m) (passive-solid cells reset: phase 0 to 1, the
// others to 0); each phase's new sum into the block partials
template <typename T>
__global__ __launch_bounds__(kBlock) void pen_ch_kernel(PenaltyArgs<T> A) {
  __shared__ double red[kBlock / kWave];
  const double rh2 = 1.0 / (A.h * A.h);
  const long sxy = (long)A.nx * A.ny;
  const double step = A.dt_ch * A.mobility;
  double acc[kMaxPhase];
  for (int m = 0; m < kMaxPhase; ++m) acc[m] = 0.0;
  for (long c = (long)blockIdx.x * kBlock + threadIdx.x; c < A.n; c += (long)gridDim.x * kBlock) {
    const int k = (int)(c / sxy);
    const long rem = c - (long)k * sxy;
    const int j = (int)(rem / A.nx), i = (int)(rem - (long)j * A.nx);
    const bool passive = A.region != nullptr && A.region[c] == 2;
    for (int m = 0; m < A.nphase; ++m) {
      double y = A.p1[(long)m * A.mstride + c] +
                 step * lap_mirror(A.mu + (long)m * A.mstride, c, i, j, k, A.nx, A.ny, A.nz, A.ndim, sxy, rh2);
      if (passive) y = m == 0 ? 1.0 : 0.0;
      const T t = (T)y;
      A.phi[(long)m * A.pstride + c] = t;
      acc[m] += (double)t;
    }
  }
  for (int m = 0; m < A.nphase; ++m) {
    const double tot = block_sum(acc[m], red);
    if (threadIdx.x == 0) A.partial[(long)m * gridDim.x + blockIdx.x] = tot;
  }
}

template <typename T>
__global__ void pen_volume_kernel(PenaltyArgs<T> A) {
  const int m = blockIdx.x;
  const double* q = A.partial + (long)m * A.nblocks;
  double s = 0.0;
  #pragma unroll 8
  for (int b = threadIdx.x; b < A.nblocks; b += kWave) s += q[b];
  s = wave_sum(s);
  if (threadIdx.x == 0) A.scal[8 * m + 4] = s / (double)A.n;
}

}  // namespace

int phase_blocks(long n) {
  long b = (n + kBlock - 1) / kBlock;
  if (b > kMaxPhaseBlocks) b = kMaxPhaseBlocks;
  return b < 1 ? 1 : (int)b;
}

template <typename T>
void launch_phase_gmax(const PhaseArgs<T>& a, hipStream_t s) {
  hipLaunchKernelGGL((gmax_kernel<T>), dim3(a.nblocks), dim3(kBlock), 0, s, a);
  hipLaunchKernelGGL(gmax_final_kernel, dim3(1), dim3(kWave), 0, s, a.partial, a.nblocks, a.scal);
}

template <typename T>
void launch_phase_step(const PhaseArgs<T>& a, hipStream_t s) {
  hipLaunchKernelGGL((step_kernel<T>), dim3(a.nblocks), dim3(kBlock), 0, s, a);
  hipLaunchKernelGGL(bracket_init_kernel, dim3(1), dim3(kWave), 0, s, a.partial, a.nblocks, a.scal, a.target);
}

template <typename T>
void launch_phase_pass(const PhaseArgs<T>& a, hipStream_t s) {
  hipLaunchKernelGGL((pass_kernel<T>), dim3(a.nblocks), dim3(kBlock), 0, s, a);
  hipLaunchKernelGGL(bracket_kernel, dim3(1), dim3(kWave), 0, s, a.partial, a.nblocks, a.scal);
}

template <typename T>
void launch_phase_apply(const PhaseArgs<T>& a, hipStream_t s) {
  hipLaunchKernelGGL((apply_kernel<T>), dim3(a.nblocks), dim3(kBlock), 0, s, a);
  hipLaunchKernelGGL(volume_final_kernel, dim3(1), dim3(kWave), 0, s, a.partial, a.nblocks, a.scal,
                     (double)a.n);
}

template <typename T>
void launch_penalty_update(const PenaltyArgs<T>& a, hipStream_t s) {
  hipLaunchKernelGGL((pen_reduce_kernel<T>), dim3(a.nblocks, a.nphase), dim3(kBlock), 0, s, a);
  hipLaunchKernelGGL((pen_final_kernel<T>), dim3(a.nphase), dim3(kWave), 0, s, a);
  hipLaunchKernelGGL((pen_p1_kernel<T>), dim3(a.nblocks), dim3(kBlock), 0, s, a);
  hipLaunchKernelGGL((pen_mu_kernel<T>), dim3(a.nblocks), dim3(kBlock), 0, s, a);
  hipLaunchKernelGGL((pen_ch_kernel<T>), dim3(a.nblocks), dim3(kBlock), 0, s, a);
  hipLaunchKernelGGL((pen_volume_kernel<T>), dim3(a.nphase), dim3(kWave), 0, s, a);
}

template void launch_penalty_update<float>(const PenaltyArgs<float>&, hipStream_t);
template void launch_penalty_update<double>(const PenaltyArgs<double>&, hipStream_t);
template void launch_phase_gmax<float>(const PhaseArgs<float>&, hipStream_t);
template void launch_phase_gmax<double>(const PhaseArgs<double>&, hipStream_t);
template void launch_phase_step<float>(const PhaseArgs<float>&, hipStream_t);
template void launch_phase_step<double>(const PhaseArgs<double>&, hipStream_t);
template void launch_phase_pass<float>(const PhaseArgs<float>&, hipStream_t);
template void launch_phase_pass<double>(const PhaseArgs<double>&, hipStream_t);
template void launch_phase_apply<float>(const PhaseArgs<float>&, hipStream_t);
template void launch_phase_apply<double>(const PhaseArgs<double>&, hipStream_t);

}  // namespace petto
