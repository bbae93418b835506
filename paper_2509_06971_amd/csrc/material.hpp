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
// E = emin + phi^p (e0 - emin).  Two solid phases with an implicit void phase
// 1 - phi1 - phi2: E = sum_m ep[m] phi_m^p (the mixture of Eq. 3.8).  Every
// fraction enters clamped to [0, 1] (the penalty update can leave the range);
// a derivative is zero where its fraction is outside.
template <typename T>
__device__ inline double modulus(const T* phi, long c, long stride, int nphase, double e0,
                                 double emin, double p, const double* ep, double* dE) {
  if (nphase == 1) {
    const double r = (double)phi[c];
    const double f = clamp01(r);
    dE[0] = p * ipow(f, p - 1.0) * (e0 - emin) * inside01(r);
    return emin + ipow(f, p) * (e0 - emin);
  }
  const double r1 = (double)phi[c], r2 = (double)phi[c + stride];
  const double f1 = clamp01(r1), f2 = clamp01(r2);
  const double rv = 1.0 - f1 - f2;
  const double fv = clamp01(rv);
  const double wv = ep[2] * ipow(fv, p - 1.0) * inside01(rv);
  dE[0] = p * (ep[0] * ipow(f1, p - 1.0) * inside01(r1) - wv);
  dE[1] = p * (ep[1] * ipow(f2, p - 1.0) * inside01(r2) - wv);
  return ep[0] * ipow(f1, p) + ep[1] * ipow(f2, p) + ep[2] * ipow(fv, p);
}

}  // namespace petto
