// Streaming bandwidth probe (a standalone program, not part of the library).
//
// What HBM and the Infinity Cache deliver to plain streaming kernels on this
// GPU, as the yardstick for the stencil kernels' measured traffic: a 256 MiB
// device copy with 16-byte accesses, and a stream with the 3D elastic sweep's
// access pattern (ten 4-byte reads and six 4-byte writes per position: u, v and
// the right-hand side in three components plus the modulus read, u and v
// written) at the positions of a 256 x 128 x 128 grid and of a grid four times
// larger.  Rates count the bytes each kernel reads and writes once.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>

#define PROBE_CHECK(x)                                                                  \
  do {                                                                                  \
    hipError_t e_ = (x);                                                                \
    if (e_ != hipSuccess) {                                                             \
      std::fprintf(stderr, "stream_probe: %s at line %d\n", hipGetErrorString(e_), __LINE__); \
      std::exit(1);                                                                     \
    }                                                                                   \
  } while (0)

__global__ void copy16(const float4* __restrict__ a, float4* __restrict__ b, long n4) {
  const long stride = (long)gridDim.x * blockDim.x;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += stride) b[i] = a[i];
}

// ten reads and six writes per position; n positions per stream
__global__ void stream10r6w(const float* __restrict__ r, float* __restrict__ w, long n) {
  const long stride = (long)gridDim.x * blockDim.x;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    float x[10];
#pragma unroll
    for (int c = 0; c < 10; ++c) x[c] = r[c * n + i];
#pragma unroll
    for (int c = 0; c < 6; ++c) w[c * n + i] = x[c] + x[c + 3] * x[9];
  }
}

template <typename F>
static float mean_ms(F launch, int reps, hipEvent_t e0, hipEvent_t e1) {
  launch();
  launch();
  PROBE_CHECK(hipEventRecord(e0));
  for (int r = 0; r < reps; ++r) launch();
  PROBE_CHECK(hipEventRecord(e1));
  PROBE_CHECK(hipEventSynchronize(e1));
  float ms = 0.f;
  PROBE_CHECK(hipEventElapsedTime(&ms, e0, e1));
  return ms / reps;
}

int main() {
  hipEvent_t e0, e1;
  PROBE_CHECK(hipEventCreate(&e0));
  PROBE_CHECK(hipEventCreate(&e1));
  {
    const long n = 64L << 20;   // floats: 256 MiB
    float *a, *b;
    PROBE_CHECK(hipMalloc(&a, n * 4));
    PROBE_CHECK(hipMalloc(&b, n * 4));
    PROBE_CHECK(hipMemset(a, 0, n * 4));
    PROBE_CHECK(hipMemset(b, 0, n * 4));
    const float ms = mean_ms([&] { copy16<<<16384, 512>>>((const float4*)a, (float4*)b, n / 4); }, 20, e0, e1);
    PROBE_CHECK(hipGetLastError());
    std::printf("copy, 256 MiB, 16-byte accesses: %.1f us, %.0f GB/s\n", ms * 1e3, 2.0 * n * 4 / (ms * 1e-3) / 1e9);
    std::fflush(stdout);
    PROBE_CHECK(hipFree(a));
    PROBE_CHECK(hipFree(b));
  }
  for (long m : {256L * 128 * 128, 4L * 256 * 128 * 128}) {
    float *r, *w;
    PROBE_CHECK(hipMalloc(&r, 10 * m * 4));
    PROBE_CHECK(hipMalloc(&w, 6 * m * 4));
    PROBE_CHECK(hipMemset(r, 0, 10 * m * 4));
    PROBE_CHECK(hipMemset(w, 0, 6 * m * 4));
    const float ms = mean_ms([&] { stream10r6w<<<16384, 256>>>(r, w, m); }, 50, e0, e1);
    PROBE_CHECK(hipGetLastError());
    std::printf("stream, 10 reads + 6 writes of 4 bytes per position, %ld positions (%.0f MB): %.1f us, %.0f GB/s\n",
                m, 16.0 * m * 4 / 1e6, ms * 1e3, 16.0 * m * 4 / (ms * 1e-3) / 1e9);
    std::fflush(stdout);
    PROBE_CHECK(hipFree(r));
    PROBE_CHECK(hipFree(w));
  }
  PROBE_CHECK(hipDeviceSynchronize());
  return 0;
}
