// Material interpolation laws (device side).
#pragma once
#include <hip/hip_runtime.h>

namespace petto {

// x^p with the common integer exponents evaluated by multiplication.
__device__ inline double ipow(double x, double p) {
  if (p == 3.0) return x * x * x;
  if (p == 2.0) return x * x;
  if (p == 1.0) return x;
  return pow(x, p);
}

__device__ inline double clamp01(double x) { return fmin(fmax(x, 0.0), 1.0); }
__device__ inline double inside01(double x) { return (x >= 0.0 && x <= 1.0) ? 1.0 : 0.0; }

// Modulus and its derivatives per stored phase.  One phase: the modified SIMP law
// E = emin + phi^p (e0 - emin).  N solid phases with an implicit void phase
// 1 - sum phi: E = sum_m ep[m] phi_m^p + ep[N] (1 - sum phi)^p (the mixture of
// Eq. 3.8).  Every fraction enters clamped to [0, 1] (the penalty update can
// leave the range); a derivative is zero where its fraction is outside.
template <typename T>
__device__ inline double modulus(const T* phi, long c, long stride, int nphase, double e0,
                                 double emin, double p, const double* ep, double* dE) {
  if (nphase == 1) {
    const double r = (double)phi[c];
    const double f = clamp01(r);
    dE[0] = p * ipow(f, p - 1.0) * (e0 - emin) * inside01(r);
    return emin + ipow(f, p) * (e0 - emin);
  }
  double sum = 0.0, E = 0.0;
  for (int m = 0; m < nphase; ++m) {
    const double r = (double)phi[c + m * stride];
    const double f = clamp01(r);
    sum += f;
    E += ep[m] * ipow(f, p);
    dE[m] = ep[m] * ipow(f, p - 1.0) * inside01(r);
  }
  const double rv = 1.0 - sum;
  const double fv = clamp01(rv);
  const double wv = ep[nphase] * ipow(fv, p - 1.0) * inside01(rv);
  for (int m = 0; m < nphase; ++m) dE[m] = p * (dE[m] - wv);
  return E + ep[nphase] * ipow(fv, p);
}

}  // namespace petto
