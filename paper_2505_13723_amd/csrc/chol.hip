// Exact block projection (Alg. 1, SAP): D = (K_BB + lambda I)^{-1} G in float64.
//
// H = s k(X_B, X_B) + lambda I is formed entry by entry, factored H = L L^T by a blocked
// right-looking Cholesky with panels of NB columns (one workgroup factors the diagonal
// block in LDS and inverts it, the rows below are multiplied by that inverse, the trailing
// lower triangle takes the rank-NB update), and G is overwritten by L^{-T} L^{-1} G with the
// same blocks (diagonal inverses applied, then the remaining rows updated).  Every reduction
// runs in a fixed order, so results are deterministic.
#include "internal.h"
#include "kfun.h"

namespace adasap {

namespace {

constexpr int NB = 64;       // panel width
constexpr int TT = 32;       // tile of the trailing update

template <int KERN>
__global__ __launch_bounds__(256) void kbb_kernel(int64_t b, int d, const void* __restrict__ X,
                                                  DT xt, const int64_t* __restrict__ B, double p,
                                                  double s, double lam, double* __restrict__ H) {
  const int64_t i = (int64_t)blockIdx.y * 16 + threadIdx.x / 16;
  const int64_t j = (int64_t)blockIdx.x * 16 + threadIdx.x % 16;
  if (i >= b || j >= b) return;
  const int64_t pi = B[i] * d, pj = B[j] * d;
  double r2 = 0.0;
  for (int f = 0; f < d; ++f) {
    const double a = xt == DT::F64 ? static_cast<const double*>(X)[pi + f]
                                   : (double)static_cast<const float*>(X)[pi + f];
    const double c = xt == DT::F64 ? static_cast<const double*>(X)[pj + f]
                                   : (double)static_cast<const float*>(X)[pj + f];
    r2 += (a - c) * (a - c);
  }
  H[i * b + j] = s * kfun<KERN, double>(r2, p) + (i == j ? lam : 0.0);
}

// factor the diagonal block H[k0:k0+nb, k0:k0+nb] = L L^T in LDS, write L back (lower) and
// its inverse to Linv (nb x nb, lower, row-major); a non-positive pivot sets sc->failed
__global__ __launch_bounds__(256) void chol_diag_kernel(int64_t b, int64_t k0, int nb,
                                                        double* __restrict__ H,
                                                        double* __restrict__ Linv,
                                                        IterScalars* __restrict__ sc) {
  __shared__ double A[NB][NB + 1];
  __shared__ double Ai[NB][NB + 1];
  const int tid = threadIdx.x;
  for (int e = tid; e < nb * nb; e += 256) {
    const int r = e / nb, c = e % nb;
    A[r][c] = c <= r ? H[(k0 + r) * b + k0 + c] : 0.0;
  }
  __syncthreads();
  for (int j = 0; j < nb; ++j) {
    if (tid == 0) {
      const double a = A[j][j];
      if (!(a > 0.0)) sc->failed = 1;
      A[j][j] = sqrt(a > 0.0 ? a : 1e-300);
    }
    __syncthreads();
    for (int r = j + 1 + tid; r < nb; r += 256) A[r][j] /= A[j][j];
    __syncthreads();
    // trailing part of the block: rows r > j, columns j < c <= r
    const int m = nb - j - 1;
    for (int e = tid; e < m * m; e += 256) {
      const int r = j + 1 + e / m, c = j + 1 + e % m;
      if (c <= r) A[r][c] -= A[r][j] * A[c][j];
    }
    __syncthreads();
  }
  // inverse of the lower factor: column c by forward substitution (one thread per column)
  if (tid < nb) {
    const int c = tid;
    for (int r = 0; r < nb; ++r) {
      double x = 0.0;
      if (r >= c) {
        double acc = r == c ? 1.0 : 0.0;
        for (int q = c; q < r; ++q) acc -= A[r][q] * Ai[q][c];
        x = acc / A[r][r];
      }
      Ai[r][c] = x;
    }
  }
  __syncthreads();
  for (int e = tid; e < nb * nb; e += 256) {
    const int r = e / nb, c = e % nb;
    if (c <= r) H[(k0 + r) * b + k0 + c] = A[r][c];
    Linv[e] = Ai[r][c];
  }
}

// rows i >= k0 + nb of the panel: L[i, k0 + c] = sum_{q <= c} H[i, k0 + q] Linv[c, q]
__global__ __launch_bounds__(256) void chol_panel_kernel(int64_t b, int64_t k0, int nb,
                                                         double* __restrict__ H,
                                                         const double* __restrict__ Linv) {
  __shared__ double Li[NB * NB];
  for (int e = threadIdx.x; e < nb * nb; e += 256) Li[e] = Linv[e];
  __syncthreads();
  const int64_t i = k0 + nb + (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= b) return;
  double a[NB];
#pragma unroll
  for (int q = 0; q < NB; ++q) a[q] = q < nb ? H[i * b + k0 + q] : 0.0;
  for (int c = 0; c < nb; ++c) {
    double acc = 0.0;
    for (int q = 0; q <= c; ++q) acc += a[q] * Li[c * nb + q];
    H[i * b + k0 + c] = acc;
  }
}

// trailing lower triangle: H[i, j] -= sum_q L[i, k0 + q] L[j, k0 + q] for k1 <= j <= i < b,
// k1 = k0 + nb; one workgroup per TT x TT tile at or below the diagonal
__global__ __launch_bounds__(256) void chol_update_kernel(int64_t b, int64_t k0, int nb,
                                                          double* __restrict__ H) {
  const int64_t k1 = k0 + nb;
  const int64_t ti = blockIdx.y, tj = blockIdx.x;
  if (tj > ti) return;
  __shared__ double Pi[TT][NB + 1], Pj[TT][NB + 1];
  const int64_t i0 = k1 + ti * TT, j0 = k1 + tj * TT;
  for (int e = threadIdx.x; e < TT * nb; e += 256) {
    const int r = e / nb, q = e % nb;
    Pi[r][q] = i0 + r < b ? H[(i0 + r) * b + k0 + q] : 0.0;
    Pj[r][q] = j0 + r < b ? H[(j0 + r) * b + k0 + q] : 0.0;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < TT * TT; e += 256) {
    const int r = e / TT, c = e % TT;
    const int64_t i = i0 + r, j = j0 + c;
    if (i >= b || j > i) continue;
    double acc = 0.0;
    for (int q = 0; q < nb; ++q) acc += Pi[r][q] * Pj[c][q];
    H[i * b + j] -= acc;
  }
}

// forward step: Y_blk = Linv_blk Y_blk (rows k0..k0+nb of the b x k right-hand side)
__global__ __launch_bounds__(256) void trsv_diag_kernel(int64_t k0, int nb, int k,
                                                        const double* __restrict__ Linv, int trans,
                                                        double* __restrict__ Y) {
  __shared__ double T[NB * 16];
  // k columns in groups of 16
  const int c0 = blockIdx.x * 16;
  for (int e = threadIdx.x; e < nb * 16; e += 256) {
    const int r = e / 16, c = c0 + e % 16;
    T[e] = c < k ? Y[(k0 + r) * k + c] : 0.0;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < nb * 16; e += 256) {
    const int r = e / 16, cc = e % 16, c = c0 + cc;
    if (c >= k) continue;
    double acc = 0.0;
    if (!trans) {
      for (int q = 0; q <= r; ++q) acc += Linv[r * nb + q] * T[q * 16 + cc];
    } else {
      for (int q = r; q < nb; ++q) acc += Linv[q * nb + r] * T[q * 16 + cc];
    }
    Y[(k0 + r) * k + c] = acc;
  }
}

// forward update: rows i >= k0 + nb: Y[i, c] -= sum_q L[i, k0 + q] Y[k0 + q, c]
// backward update: rows i < k0: Y[i, c] -= sum_q L[k0 + q, i] Y[k0 + q, c]
__global__ __launch_bounds__(256) void trsv_update_kernel(int64_t b, int64_t k0, int nb, int k,
                                                          const double* __restrict__ H, int back,
                                                          double* __restrict__ Y) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t rows = back ? k0 : b - k0 - nb;
  if (e >= rows * k) return;
  const int64_t i = (back ? 0 : k0 + nb) + e / k;
  const int c = (int)(e % k);
  double acc = 0.0;
  for (int q = 0; q < nb; ++q) {
    const double l = back ? H[(k0 + q) * b + i] : H[i * b + k0 + q];
    acc += l * Y[(k0 + q) * k + c];
  }
  Y[i * k + c] -= acc;
}

__global__ void unit_step_kernel(IterScalars* sc, double lam) {
  sc->eta = 1.0;
  sc->lam_hat = 1.0;
  sc->rho = lam;
  sc->delta = 0.0;
  sc->sweeps = 0;
  sc->not_pd = 0;
  sc->failed = 0;
}

}  // namespace

size_t exact_linv_doubles(int64_t b) { return (size_t)((b + NB - 1) / NB) * NB * NB; }

adasap_status_t exact_factor(int kern, double ell, double outputscale, double lam, int64_t b, int d,
                             const void* X, DT xt, const int64_t* B, double* H, double* Linv,
                             IterScalars* sc, hipStream_t s) {
  const dim3 g16((unsigned)((b + 15) / 16), (unsigned)((b + 15) / 16));
  const double p = kernel_param(kern, ell);
  switch (kern) {
    case ADASAP_RBF:
      hipLaunchKernelGGL(kbb_kernel<ADASAP_RBF>, g16, dim3(256), 0, s, b, d, X, xt, B, p, outputscale, lam, H);
      break;
    case ADASAP_MATERN12:
      hipLaunchKernelGGL(kbb_kernel<ADASAP_MATERN12>, g16, dim3(256), 0, s, b, d, X, xt, B, p, outputscale, lam, H);
      break;
    case ADASAP_MATERN32:
      hipLaunchKernelGGL(kbb_kernel<ADASAP_MATERN32>, g16, dim3(256), 0, s, b, d, X, xt, B, p, outputscale, lam, H);
      break;
    default:
      hipLaunchKernelGGL(kbb_kernel<ADASAP_MATERN52>, g16, dim3(256), 0, s, b, d, X, xt, B, p, outputscale, lam, H);
      break;
  }
  ADASAP_LAUNCH_CHECK();
  hipLaunchKernelGGL(unit_step_kernel, dim3(1), dim3(1), 0, s, sc, lam);
  ADASAP_LAUNCH_CHECK();
  for (int64_t k0 = 0, blk = 0; k0 < b; k0 += NB, ++blk) {
    const int nb = (int)(b - k0 < NB ? b - k0 : NB);
    double* Li = Linv + blk * NB * NB;
    hipLaunchKernelGGL(chol_diag_kernel, dim3(1), dim3(256), 0, s, b, k0, nb, H, Li, sc);
    ADASAP_LAUNCH_CHECK();
    const int64_t rest = b - k0 - nb;
    if (rest <= 0) break;
    hipLaunchKernelGGL(chol_panel_kernel, dim3((unsigned)((rest + 255) / 256)), dim3(256), 0, s, b,
                       k0, nb, H, Li);
    ADASAP_LAUNCH_CHECK();
    const unsigned tiles = (unsigned)((rest + TT - 1) / TT);
    hipLaunchKernelGGL(chol_update_kernel, dim3(tiles, tiles), dim3(256), 0, s, b, k0, nb, H);
    ADASAP_LAUNCH_CHECK();
  }
  return ADASAP_OK;
}

adasap_status_t exact_solve(int64_t b, int k, const double* H, const double* Linv, double* Y,
                            hipStream_t s) {
  const unsigned cg = (unsigned)((k + 15) / 16);
  // Y <- L^{-1} Y
  for (int64_t k0 = 0, blk = 0; k0 < b; k0 += NB, ++blk) {
    const int nb = (int)(b - k0 < NB ? b - k0 : NB);
    hipLaunchKernelGGL(trsv_diag_kernel, dim3(cg), dim3(256), 0, s, k0, nb, k, Linv + blk * NB * NB,
                       0, Y);
    ADASAP_LAUNCH_CHECK();
    const int64_t rest = (b - k0 - nb) * k;
    if (rest > 0) {
      hipLaunchKernelGGL(trsv_update_kernel, dim3((unsigned)((rest + 255) / 256)), dim3(256), 0, s, b,
                         k0, nb, k, H, 0, Y);
      ADASAP_LAUNCH_CHECK();
    }
  }
  // Y <- L^{-T} Y, last block first
  const int64_t nblk = (b + NB - 1) / NB;
  for (int64_t blk = nblk - 1; blk >= 0; --blk) {
    const int64_t k0 = blk * NB;
    const int nb = (int)(b - k0 < NB ? b - k0 : NB);
    hipLaunchKernelGGL(trsv_diag_kernel, dim3(cg), dim3(256), 0, s, k0, nb, k, Linv + blk * NB * NB,
                       1, Y);
    ADASAP_LAUNCH_CHECK();
    const int64_t rest = k0 * k;
    if (rest > 0) {
      hipLaunchKernelGGL(trsv_update_kernel, dim3((unsigned)((rest + 255) / 256)), dim3(256), 0, s, b,
                         k0, nb, k, H, 1, Y);
      ADASAP_LAUNCH_CHECK();
    }
  }
  return ADASAP_OK;
}

}  // namespace adasap
