// Covariance functions evaluated from a squared distance, shared by the kernel-block
// products.  Parameters are pre-folded on the host so each evaluation is a handful of
// instructions:
//   RBF        exp(-r2/(2 ell^2))       = exp2(r2 * p),   p = -log2(e)/(2 ell^2)
//   Matern-1/2 exp(-r/ell)              = exp2(-a log2 e), a = r/ell
//   Matern-3/2 (1+a) exp(-a),             a = sqrt(3) r/ell
//   Matern-5/2 (1+a+a^2/3) exp(-a),       a = sqrt(5) r/ell
// For the Matern family p is the factor turning r into a.
#pragma once

#include <hip/hip_runtime.h>

#include "../../include/adasap.h"

namespace adasap {

constexpr double LOG2E = 1.4426950408889634;

inline double kernel_param(int kern, double ell) {
  switch (kern) {
    case ADASAP_RBF: return -LOG2E / (2.0 * ell * ell);
    case ADASAP_MATERN12: return 1.0 / ell;
    case ADASAP_MATERN32: return 1.7320508075688772 / ell;
    default: return 2.23606797749979 / ell;
  }
}

__device__ inline double exp2_t(double x) { return exp2(x); }
__device__ inline float exp2_t(float x) { return exp2f(x); }
__device__ inline double sqrt_t(double x) { return sqrt(x); }
__device__ inline float sqrt_t(float x) { return sqrtf(x); }

template <int KERN, typename T>
__device__ inline T kfun(T r2, T p) {
  if constexpr (KERN == ADASAP_RBF) {
    return exp2_t(r2 * p);
  } else {
    T r = sqrt_t(r2 > T(0) ? r2 : T(0));
    T a = r * p;
    T e = exp2_t(-a * T(LOG2E));
    if constexpr (KERN == ADASAP_MATERN12) return e;
    else if constexpr (KERN == ADASAP_MATERN32) return (T(1) + a) * e;
    else return (T(1) + a + a * a * T(1.0 / 3.0)) * e;
  }
}

}  // namespace adasap
