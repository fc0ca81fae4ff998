// Shared definitions of the ADASAP HIP library (gfx950): error plumbing, the
// Philox4x64-10 counter-based generator, per-solve device scalars.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "../../include/adasap.h"

namespace adasap {

// ---- errors ------------------------------------------------------------------------------

void set_error(const std::string& msg);

struct Status {
  adasap_status_t code = ADASAP_OK;
};

#define ADASAP_HIP(call)                                                                 \
  do {                                                                                   \
    hipError_t e_ = (call);                                                              \
    if (e_ != hipSuccess) {                                                              \
      ::adasap::set_error(std::string("HIP error ") + hipGetErrorString(e_) + " at " +   \
                          __FILE__ + ":" + std::to_string(__LINE__) + " (" #call ")");   \
      return ADASAP_ERR_DEVICE;                                                          \
    }                                                                                    \
  } while (0)

#define ADASAP_TRY(expr)                         \
  do {                                           \
    adasap_status_t s_ = (expr);                 \
    if (s_ != ADASAP_OK) return s_;              \
  } while (0)

#define ADASAP_LAUNCH_CHECK() ADASAP_HIP(hipGetLastError())

// ---- Philox4x64-10 (Salmon et al., SC'11) ------------------------------------------------
// Stream (seed, purpose, t): key = (seed, purpose); block i has counter (i + 1, t, 0, 0)
// and yields its four 64-bit words in order.

struct u64x4 {
  uint64_t v[4];
};

__host__ __device__ inline uint64_t mulhi64(uint64_t a, uint64_t b) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __umul64hi(a, b);
#else
  return (uint64_t)(((unsigned __int128)a * (unsigned __int128)b) >> 64);
#endif
}

__host__ __device__ inline u64x4 philox4x64_10(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3,
                                               uint64_t k0, uint64_t k1) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    uint64_t hi0 = mulhi64(M0, c0), lo0 = M0 * c0;
    uint64_t hi1 = mulhi64(M1, c2), lo1 = M1 * c2;
    uint64_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
    k0 += W0;
    k1 += W1;
  }
  u64x4 o;
  o.v[0] = c0;
  o.v[1] = c1;
  o.v[2] = c2;
  o.v[3] = c3;
  return o;
}

// ---- random-draw purposes (second key word) -----------------------------------------------
constexpr uint64_t PURPOSE_B = 5;
constexpr uint64_t PURPOSE_OMEGA = 6;
constexpr uint64_t PURPOSE_POW = 7;
constexpr uint64_t PURPOSE_MINIBATCH = 11;  // warm-start training order, epoch = t
constexpr uint64_t PURPOSE_RESROWS = 12;    // rows of a subsampled residual estimate
constexpr uint64_t PURPOSE_SWEEP_STRIDE = 16;

// ---- device-resident scalars of one iteration (never copied back inside the loop) -----------
struct IterScalars {
  double delta;       // Nystrom shift actually used
  double rho;         // damping
  double lam_hat;     // Rayleigh quotient of the last powering application
  double eta;         // step size 1 / lam_hat
  double vnorm2;      // scratch: squared norm for the powering normalisation
  double rq;          // scratch: Rayleigh quotient numerator
  int32_t sweeps;     // Jacobi sweeps performed
  int32_t not_pd;     // 1 if the Cholesky of the Nystrom core needed a larger shift
  int32_t failed;     // 1 if it failed after every retry
  int32_t pad;
};

}  // namespace adasap
