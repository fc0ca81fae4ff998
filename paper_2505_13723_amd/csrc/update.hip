// Gathers of the block rows and the accelerated update of Alg. NestAcc.
//
// With D = P_B^{-1} G and the step eta, the update
//   W_{t+1} = Z_t - eta I_B^T D
//   V_{t+1} = beta V_t + (1 - beta) Z_t - gamma eta I_B^T D
//   Z_{t+1} = alpha V_{t+1} + (1 - alpha) W_{t+1}
// is a fixed 2x2 map on (V, Z) for every row plus a correction on the b rows of B, so it
// runs as one streaming pass over all n rows followed by a pass over the block rows.
#include "internal.h"

namespace adasap {

namespace {

template <typename T>
__device__ inline double ldd(const void* p, int64_t i) {
  return (double)static_cast<const T*>(p)[i];
}

__device__ inline double ld_dt(const void* p, DT t, int64_t i) {
  switch (t) {
    case DT::F64: return static_cast<const double*>(p)[i];
    case DT::F32: return (double)static_cast<const float*>(p)[i];
    default: return (double)(float)static_cast<const _Float16*>(p)[i];
  }
}

__device__ inline void st_dt(void* p, DT t, int64_t i, double v) {
  switch (t) {
    case DT::F64: static_cast<double*>(p)[i] = v; break;
    case DT::F32: static_cast<float*>(p)[i] = (float)v; break;
    default: static_cast<_Float16*>(p)[i] = (_Float16)(float)v; break;
  }
}

__global__ void gather_kernel(int64_t rows, int cols, const void* __restrict__ src, DT st,
                              int64_t lds, const int64_t* __restrict__ idx, void* __restrict__ dst,
                              DT dt, int64_t ldd_) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= rows * cols) return;
  const int64_t i = e / cols;
  const int c = (int)(e % cols);
  st_dt(dst, dt, i * ldd_ + c, ld_dt(src, st, idx[i] * lds + c));
}

__global__ void convert_kernel(int64_t count, const void* __restrict__ src, DT st,
                               void* __restrict__ dst, DT dt) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) st_dt(dst, dt, i, ld_dt(src, st, i));
}

template <typename T>
__global__ void nesterov_dense_kernel(int64_t count, T* __restrict__ V, T* __restrict__ Z,
                                      double beta, double alpha, int z_next, void* __restrict__ W,
                                      DT wt, const int32_t* __restrict__ row_prob,
                                      const double* __restrict__ coefs, int k) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  if (row_prob) {
    // batch: (beta, gamma, alpha) of the problem owning this row
    const int pb = row_prob[i / k];
    beta = coefs[3 * pb];
    alpha = coefs[3 * pb + 2];
  }
  const double v = (double)V[i], z = (double)Z[i];
  if (W) st_dt(W, wt, i, z);
  const double vn = beta * v + (1.0 - beta) * z;
  const double zn = alpha * (z_next ? vn : v) + (1.0 - alpha) * z;
  V[i] = (T)vn;
  Z[i] = (T)zn;
}

template <typename T>
__global__ void nesterov_sparse_kernel(int64_t b, int k, const int64_t* __restrict__ B,
                                       const double* __restrict__ D, T* __restrict__ V,
                                       T* __restrict__ Z, double gamma, double alpha, int accel,
                                       int z_next, const IterScalars* __restrict__ sc,
                                       void* __restrict__ W, DT wt,
                                       const double* __restrict__ coefs) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= b * k) return;
  // batch: problem blockIdx.y has its block, direction and scalars b*k apart
  const int pb = blockIdx.y;
  B += (int64_t)pb * b;
  D += (int64_t)pb * b * k;
  sc += pb;
  if (coefs) {
    gamma = coefs[3 * pb + 1];
    alpha = coefs[3 * pb + 2];
  }
  const int64_t i = e / k;
  const int c = (int)(e % k);
  const int64_t g = B[i] * k + c;
  const double step = sc->eta * D[e];
  if (!accel) {
    Z[g] = (T)((double)Z[g] - step);
    return;
  }
  V[g] = (T)((double)V[g] - gamma * step);
  const double zc = z_next ? (alpha * gamma + 1.0 - alpha) : (1.0 - alpha);
  Z[g] = (T)((double)Z[g] - zc * step);
  if (W) st_dt(W, wt, g, ld_dt(W, wt, g) - step);
}

__global__ void accumulate_kernel(int64_t count, const void* __restrict__ W, DT wt,
                                  double* __restrict__ acc) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) acc[i] += ld_dt(W, wt, i);
}

__global__ void scale_store_kernel(int64_t count, const double* __restrict__ src, double scale,
                                   void* __restrict__ dst, DT dt) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) st_dt(dst, dt, i, scale * src[i]);
}

__global__ void nonfinite_kernel(int64_t count, const void* __restrict__ src, DT st,
                                 int* __restrict__ flag) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) {
    const double v = ld_dt(src, st, i);
    if (!isfinite(v)) atomicOr(flag, 1);
  }
}

__global__ void add_kernel(int64_t count, void* __restrict__ a, DT at, const void* __restrict__ b,
                           DT bt) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) st_dt(a, at, i, ld_dt(a, at, i) + ld_dt(b, bt, i));
}

inline unsigned nblocks(int64_t count) { return (unsigned)((count + 255) / 256); }

}  // namespace

adasap_status_t gather_rows(int64_t rows, int cols, const void* src, DT st, int64_t lds,
                            const int64_t* idx, void* dst, DT dt, int64_t ldd_, hipStream_t s) {
  if (rows * cols <= 0) return ADASAP_OK;
  hipLaunchKernelGGL(gather_kernel, dim3(nblocks(rows * cols)), dim3(256), 0, s, rows, cols, src,
                     st, lds, idx, dst, dt, ldd_);
  ADASAP_LAUNCH_CHECK();
  return ADASAP_OK;
}

// out[i, j] = X[i, j] * scale[j] in float64 (per-coordinate lengthscales folded into the points)
__global__ void scale_columns_kernel(int64_t n, int d, const void* __restrict__ X, DT xt,
                                     const double* __restrict__ scale, double* __restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * d) return;
  const double x = xt == DT::F64 ? static_cast<const double*>(X)[e]
                                 : (double)static_cast<const float*>(X)[e];
  out[e] = x * scale[e % d];
}

adasap_status_t scale_columns(int64_t n, int d, const void* X, DT xt, const double* scale,
                              double* out, hipStream_t s) {
  if (n * d <= 0) return ADASAP_OK;
  hipLaunchKernelGGL(scale_columns_kernel, dim3(nblocks(n * d)), dim3(256), 0, s, n, d, X, xt, scale,
                     out);
  ADASAP_LAUNCH_CHECK();
  return ADASAP_OK;
}

adasap_status_t convert(int64_t count, const void* src, DT st, void* dst, DT dt, hipStream_t s) {
  if (count <= 0) return ADASAP_OK;
  hipLaunchKernelGGL(convert_kernel, dim3(nblocks(count)), dim3(256), 0, s, count, src, st, dst, dt);
  ADASAP_LAUNCH_CHECK();
  return ADASAP_OK;
}

adasap_status_t nesterov_dense(int64_t count, void* V, void* Z, DT st, const NestCoef& c,
                               void* Wout, DT wt, hipStream_t s, const int32_t* row_prob,
                               const double* coefs, int k) {
  if (count <= 0) return ADASAP_OK;
  if (st == DT::F64)
    hipLaunchKernelGGL(nesterov_dense_kernel<double>, dim3(nblocks(count)), dim3(256), 0, s, count,
                       static_cast<double*>(V), static_cast<double*>(Z), c.beta, c.alpha,
                       c.z_uses_v_next, Wout, wt, row_prob, coefs, k);
  else
    hipLaunchKernelGGL(nesterov_dense_kernel<float>, dim3(nblocks(count)), dim3(256), 0, s, count,
                       static_cast<float*>(V), static_cast<float*>(Z), c.beta, c.alpha,
                       c.z_uses_v_next, Wout, wt, row_prob, coefs, k);
  ADASAP_LAUNCH_CHECK();
  return ADASAP_OK;
}

adasap_status_t nesterov_sparse(int64_t b, int k, const int64_t* B, const double* D, void* V,
                                void* Z, DT st, const NestCoef& c, const IterScalars* sc,
                                void* Wout, DT wt, hipStream_t s, int P, const double* coefs) {
  const int64_t count = b * k;
  if (count <= 0) return ADASAP_OK;
  if (st == DT::F64)
    hipLaunchKernelGGL(nesterov_sparse_kernel<double>, dim3(nblocks(count), P), dim3(256), 0, s, b,
                       k, B, D, static_cast<double*>(V), static_cast<double*>(Z), c.gamma, c.alpha,
                       c.accel, c.z_uses_v_next, sc, Wout, wt, coefs);
  else
    hipLaunchKernelGGL(nesterov_sparse_kernel<float>, dim3(nblocks(count), P), dim3(256), 0, s, b,
                       k, B, D, static_cast<float*>(V), static_cast<float*>(Z), c.gamma, c.alpha,
                       c.accel, c.z_uses_v_next, sc, Wout, wt, coefs);
  ADASAP_LAUNCH_CHECK();
  return ADASAP_OK;
}

adasap_status_t add_inplace(int64_t count, void* a, DT at, const void* b, DT bt, hipStream_t s) {
  if (count <= 0) return ADASAP_OK;
  hipLaunchKernelGGL(add_kernel, dim3(nblocks(count)), dim3(256), 0, s, count, a, at, b, bt);
  ADASAP_LAUNCH_CHECK();
  return ADASAP_OK;
}

adasap_status_t accumulate(int64_t count, const void* W, DT wt, double* acc, hipStream_t s) {
  if (count <= 0) return ADASAP_OK;
  hipLaunchKernelGGL(accumulate_kernel, dim3(nblocks(count)), dim3(256), 0, s, count, W, wt, acc);
  ADASAP_LAUNCH_CHECK();
  return ADASAP_OK;
}

adasap_status_t scale_store(int64_t count, const double* src, double scale, void* dst, DT dt,
                            hipStream_t s) {
  if (count <= 0) return ADASAP_OK;
  hipLaunchKernelGGL(scale_store_kernel, dim3(nblocks(count)), dim3(256), 0, s, count, src, scale,
                     dst, dt);
  ADASAP_LAUNCH_CHECK();
  return ADASAP_OK;
}

adasap_status_t any_nonfinite(int64_t count, const void* src, DT st, int* flag, DevBuf& tmp,
                              hipStream_t s) {
  ADASAP_TRY(tmp.ensure(sizeof(int)));
  ADASAP_HIP(hipMemsetAsync(tmp.p, 0, sizeof(int), s));
  if (count > 0) {
    hipLaunchKernelGGL(nonfinite_kernel, dim3(nblocks(count)), dim3(256), 0, s, count, src, st,
                       tmp.as<int>());
    ADASAP_LAUNCH_CHECK();
  }
  ADASAP_HIP(hipMemcpyAsync(flag, tmp.p, sizeof(int), hipMemcpyDeviceToHost, s));
  ADASAP_HIP(hipStreamSynchronize(s));
  return ADASAP_OK;
}

}  // namespace adasap
