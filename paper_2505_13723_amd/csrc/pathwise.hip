// Pathwise posterior samples and predictive metrics (Sec. 2.1 pathwise conditioning; the
// test RMSE and mean negative log-likelihood of Sec. 5.1).
//
// With W = [W_0 | W_1 .. W_S] solving (K + lambda I) W = [y | f_s(X) + zeta_s] and
// P = k(X*, X) W (one kernel-block product), column 0 of P is the posterior mean and
// sample s is f_s(X*) + P_0 - P_s.  The metrics reduce per test point, then add the
// per-block partial sums in a fixed order (deterministic).
#include <cmath>

#include "internal.h"

namespace adasap {

namespace {

__device__ inline double ldv(const void* p, DT t, int64_t i) {
  return t == DT::F64 ? static_cast<const double*>(p)[i] : (double)static_cast<const float*>(p)[i];
}

__device__ inline void stv(void* p, DT t, int64_t i, double v) {
  if (t == DT::F64) static_cast<double*>(p)[i] = v;
  else static_cast<float*>(p)[i] = (float)v;
}

// out[i, s] = prior[i, s - 1] + out[i, 0] - out[i, s] for s >= 1 (out holds k(X*, X) W)
__global__ void pathwise_combine_kernel(int64_t m, int k, const void* __restrict__ prior, DT pt,
                                        void* __restrict__ out, DT ot) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t cols = k - 1;
  if (e >= m * cols) return;
  const int64_t i = e / cols;
  const int s = 1 + (int)(e % cols);
  const double v = ldv(prior, pt, i * cols + s - 1) + ldv(out, ot, i * k) - ldv(out, ot, i * k + s);
  stv(out, ot, i * k + s, v);
}

constexpr int PM_ROWS = 1024;

// per block of PM_ROWS test points: sum (mu - y)^2 and sum of the Gaussian NLL terms
__global__ __launch_bounds__(256) void metrics_partial_kernel(int64_t m, int k,
                                                              const void* __restrict__ smp,
                                                              const void* __restrict__ ys, DT t,
                                                              double lam, double* __restrict__ part) {
  __shared__ double r1[256], r2[256];
  const int64_t i0 = (int64_t)blockIdx.x * PM_ROWS;
  const int64_t i1 = i0 + PM_ROWS < m ? i0 + PM_ROWS : m;
  double se = 0.0, nl = 0.0;
  for (int64_t i = i0 + threadIdx.x; i < i1; i += 256) {
    const double mu = ldv(smp, t, i * k);
    const double y = ldv(ys, t, i);
    double v = 0.0;
    for (int s = 1; s < k; ++s) {
      const double dv = ldv(smp, t, i * k + s) - mu;
      v += dv * dv;
    }
    if (k > 1) v /= (double)(k - 1);
    const double var = v + lam;
    const double r = y - mu;
    se += r * r;
    nl += 0.5 * log(2.0 * M_PI * var) + r * r / (2.0 * var);
  }
  r1[threadIdx.x] = se;
  r2[threadIdx.x] = nl;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) {
      r1[threadIdx.x] += r1[threadIdx.x + h];
      r2[threadIdx.x] += r2[threadIdx.x + h];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = r1[0];
    part[2 * blockIdx.x + 1] = r2[0];
  }
}

__global__ void metrics_final_kernel(const double* __restrict__ part, int nblk, int64_t m,
                                     double* __restrict__ out) {
  if (threadIdx.x == 0) {
    double se = 0.0, nl = 0.0;
    for (int b = 0; b < nblk; ++b) {
      se += part[2 * b];
      nl += part[2 * b + 1];
    }
    out[0] = sqrt(se / (double)m);
    out[1] = nl / (double)m;
  }
}

// per column c and block of rows: the first row of the largest value (NaN never wins)
__global__ __launch_bounds__(256) void argmax_partial_kernel(int64_t m, int k, int64_t ld,
                                                             const void* __restrict__ a, DT t,
                                                             int64_t rows_per_blk,
                                                             double* __restrict__ pv,
                                                             int64_t* __restrict__ pi) {
  __shared__ double bv[256];
  __shared__ int64_t bi[256];
  const int c = blockIdx.y;
  const int64_t r0 = (int64_t)blockIdx.x * rows_per_blk;
  const int64_t r1 = r0 + rows_per_blk < m ? r0 + rows_per_blk : m;
  double best = -INFINITY;
  int64_t arg = -1;
  for (int64_t i = r0 + threadIdx.x; i < r1; i += 256) {
    const double v = ldv(a, t, i * ld + c);
    if (v > best) {
      best = v;
      arg = i;
    }
  }
  bv[threadIdx.x] = best;
  bi[threadIdx.x] = arg;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) {
      const double v2 = bv[threadIdx.x + h];
      const int64_t i2 = bi[threadIdx.x + h];
      if (i2 >= 0 && (bi[threadIdx.x] < 0 || v2 > bv[threadIdx.x] ||
                      (v2 == bv[threadIdx.x] && i2 < bi[threadIdx.x]))) {
        bv[threadIdx.x] = v2;
        bi[threadIdx.x] = i2;
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    pv[(int64_t)c * gridDim.x + blockIdx.x] = bv[0];
    pi[(int64_t)c * gridDim.x + blockIdx.x] = bi[0];
  }
}

__global__ void argmax_final_kernel(int nblk, int k, const double* __restrict__ pv,
                                    const int64_t* __restrict__ pi, int64_t* __restrict__ out) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= k) return;
  double best = -INFINITY;
  int64_t arg = -1;
  for (int b = 0; b < nblk; ++b) {
    const int64_t i = pi[(int64_t)c * nblk + b];
    const double v = pv[(int64_t)c * nblk + b];
    if (i >= 0 && (arg < 0 || v > best)) {
      best = v;
      arg = i;
    }
  }
  out[c] = arg;
}

}  // namespace

adasap_status_t pathwise_combine(int64_t m, int k, const void* prior, DT pt, void* out, DT ot,
                                 hipStream_t s) {
  const int64_t count = m * (k - 1);
  if (count <= 0) return ADASAP_OK;
  hipLaunchKernelGGL(pathwise_combine_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s,
                     m, k, prior, pt, out, ot);
  ADASAP_LAUNCH_CHECK();
  return ADASAP_OK;
}

}  // namespace adasap

using namespace adasap;

extern "C" adasap_status_t adasap_predictive_metrics(int64_t m, int32_t k, const void* samples,
                                                     const void* ystar, double lambda, int32_t dtype,
                                                     void* stream, double* rmse, double* nll) {
  if (m < 1 || k < 1) {
    set_error("need m >= 1 and k >= 1");
    return ADASAP_ERR_INVALID_ARG;
  }
  if (!samples || !ystar) {
    set_error("samples and ystar must be non-null device pointers");
    return ADASAP_ERR_INVALID_ARG;
  }
  if (!(lambda >= 0) || !std::isfinite(lambda)) {
    set_error("lambda must be finite and >= 0");
    return ADASAP_ERR_INVALID_ARG;
  }
  if (dtype != ADASAP_DTYPE_F32 && dtype != ADASAP_DTYPE_F64) {
    set_error("unknown dtype");
    return ADASAP_ERR_INVALID_ARG;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  const DT t = dtype == ADASAP_DTYPE_F64 ? DT::F64 : DT::F32;
  const int nblk = (int)((m + PM_ROWS - 1) / PM_ROWS);
  DevBuf part, res;
  ADASAP_TRY(part.ensure((size_t)nblk * 2 * sizeof(double)));
  ADASAP_TRY(res.ensure(2 * sizeof(double)));
  hipLaunchKernelGGL(metrics_partial_kernel, dim3(nblk), dim3(256), 0, s, m, k, samples, ystar, t,
                     lambda, part.as<double>());
  ADASAP_LAUNCH_CHECK();
  hipLaunchKernelGGL(metrics_final_kernel, dim3(1), dim3(64), 0, s, part.as<double>(), nblk, m,
                     res.as<double>());
  ADASAP_LAUNCH_CHECK();
  double h[2];
  ADASAP_HIP(hipMemcpyAsync(h, res.p, sizeof(h), hipMemcpyDeviceToHost, s));
  ADASAP_HIP(hipStreamSynchronize(s));
  if (rmse) *rmse = h[0];
  if (nll) *nll = h[1];
  return ADASAP_OK;
}

extern "C" adasap_status_t adasap_column_argmax(int64_t m, int32_t k, int64_t ld, const void* a,
                                                int32_t dtype, void* stream, int64_t* out) {
  if (m < 1 || k < 1 || ld < k) {
    set_error("need m >= 1, k >= 1 and ld >= k");
    return ADASAP_ERR_INVALID_ARG;
  }
  if (!a || !out) {
    set_error("a and out must be non-null device pointers");
    return ADASAP_ERR_INVALID_ARG;
  }
  if (dtype != ADASAP_DTYPE_F32 && dtype != ADASAP_DTYPE_F64) {
    set_error("unknown dtype");
    return ADASAP_ERR_INVALID_ARG;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  const DT t = dtype == ADASAP_DTYPE_F64 ? DT::F64 : DT::F32;
  int64_t rpb = (m + 255) / 256;
  if (rpb < 1024) rpb = 1024;
  const int nblk = (int)((m + rpb - 1) / rpb);
  DevBuf pv, pi;
  ADASAP_TRY(pv.ensure((size_t)nblk * k * sizeof(double)));
  ADASAP_TRY(pi.ensure((size_t)nblk * k * sizeof(int64_t)));
  hipLaunchKernelGGL(argmax_partial_kernel, dim3(nblk, k), dim3(256), 0, s, m, k, ld, a, t, rpb,
                     pv.as<double>(), pi.as<int64_t>());
  ADASAP_LAUNCH_CHECK();
  hipLaunchKernelGGL(argmax_final_kernel, dim3((k + 127) / 128), dim3(128), 0, s, nblk, k,
                     pv.as<double>(), pi.as<int64_t>(), out);
  ADASAP_LAUNCH_CHECK();
  ADASAP_HIP(hipStreamSynchronize(s));
  return ADASAP_OK;
}
