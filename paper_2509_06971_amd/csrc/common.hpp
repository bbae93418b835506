// Shared definitions of the HIP kernels and the host library (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace petto {

constexpr int kBlock = 256;         // threads per workgroup for every stencil kernel
constexpr int kWave = 64;           // CDNA wavefront width
constexpr int kNumXcd = 8;          // MI355X accelerator complex dies (one L2 each)
constexpr int kMaxDesigns = 1024;   // upper bound of a batch
constexpr int kCand = 63;           // candidate shifts per volume-bracket pass
constexpr int kRing = 8;             // status ring slots polled by the host
constexpr int kMaxPhase = 6;         // stored solid phases (PETTO_MAX_PHASES)

// Solve bookkeeping of one design, resident in device memory.  Written by the
// setup / finalize kernels, read by every sweep (coefficients, stop flag).
struct SolveState {
  double dt, a, c;        // v <- a v + c r,  u <- u + dt v   (c folds 1/h^d)
  double fnorm;           // ||F|| (inner correction solves: ||b||)
  double tol;             // absolute stop level on ||r|| is tol * fnorm
  double rho, rho_first;
  double r_pde;
  double sumsq;           // sum r^2 of the last check
  double theta;
  double hd;              // h^d
  double dt_scale;        // automatic step: dt = dt_scale * sqrt(theta)
  double theta_min;       // adaptive damping never goes below this
  int32_t iters, done, status, checks;
  int32_t max_iter, check_every, replay, first_seen;
  int32_t adapt, pad2, pad3, pad4;
};

// State-layout range and uniform source of one design (Rayleigh-quotient sums).
struct StateRange {
  long off;
  long n;
  double fsrc;            // used when the dense load is absent
};

// What the host polls after each block of sweeps (one ring slot per block).
struct PollRecord {
  int32_t all_done;
  int32_t any_diverged;
  int32_t any_not_converged;
  int32_t seq;
};

// Wave-level sum of a double through cross-lane shuffles (wave64).
__device__ inline double wave_sum(double x) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, kWave);
  return x;
}

__device__ inline double wave_max(double x) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) x = fmax(x, __shfl_xor(x, off, kWave));
  return x;
}

__device__ inline double wave_min(double x) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) x = fmin(x, __shfl_xor(x, off, kWave));
  return x;
}

// Block-level sum in a fixed order (waves, then lanes): deterministic.
__device__ inline double block_sum(double x, double* sh /* >= kBlock/kWave */) {
  x = wave_sum(x);
  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
  if (lane == 0) sh[w] = x;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0) {
    for (int i = 0; i < (int)(blockDim.x / kWave); ++i) s += sh[i];
  }
  __syncthreads();
  return s;  // valid in thread 0
}

__device__ inline double block_max(double x, double* sh) {
  x = wave_max(x);
  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
  if (lane == 0) sh[w] = x;
  __syncthreads();
  double s = -INFINITY;
  if (threadIdx.x == 0) {
    for (int i = 0; i < (int)(blockDim.x / kWave); ++i) s = fmax(s, sh[i]);
  }
  __syncthreads();
  return s;
}

__device__ inline double block_min(double x, double* sh) {
  x = wave_min(x);
  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
  if (lane == 0) sh[w] = x;
  __syncthreads();
  double s = INFINITY;
  if (threadIdx.x == 0) {
    for (int i = 0; i < (int)(blockDim.x / kWave); ++i) s = fmin(s, sh[i]);
  }
  __syncthreads();
  return s;
}

// Workgroups are dealt to the XCDs round-robin (block b runs on XCD b mod 8).
// Give each XCD a contiguous range of tiles so neighbouring tiles, which share
// halos, meet in the same L2.  A bijection of [0, nb).
__device__ inline int xcd_tile(int b, int nb) {
  const int q = nb / kNumXcd, r = nb % kNumXcd;
  const int x = b % kNumXcd, k = b / kNumXcd;
  return x * q + (x < r ? x : r) + k;
}

}  // namespace petto
