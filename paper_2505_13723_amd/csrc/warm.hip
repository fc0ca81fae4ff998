// Learned warm start on gfx950: random Fourier features, the RFF ridge mean, and the
// training (forward, backward, Adam) and inference of the dense SiLU network that predicts
// the posterior mean m = y - lambda W* of a problem from its points (the initial iterate of
// Alg. 2 is then W_0 = (y - m^) / lambda).
//
// Network input row of a point: [cos(Omega x + c) (D) | y | m_rff] (D + 2 floats).
// Ridge mean: phi = sqrt(2/D) cos(Omega x + c), theta = (Phi^T Phi + lambda I)^{-1} Phi^T y
// over the problem's own points; the Gram matrix [cos | y]^T [cos | y] is accumulated in
// float64 by tiled partial sums added in a fixed order, and factored by a one-workgroup
// Cholesky in float64.
// Dense layers: float32 tiled GEMM on the vector ALUs (64 x 64 output tiles, 16-deep LDS
// stages); SiLU and its derivative fused into the GEMM epilogues.
#include <cmath>
#include <cstring>
#include <vector>

#include "../../include/adasap_warm.h"
#include "internal.h"

using namespace adasap;

struct adasap_ws_s {
  adasap_ws_config_t cfg{};
  hipStream_t s = nullptr;
  int64_t np = 0;
  int64_t offW[4] = {0, 0, 0, 0}, offB[4] = {0, 0, 0, 0};
  DevBuf freqs, phases, params, grad, adam_m, adam_v;
  int64_t adam_t = 0;
  DevBuf trainA, traint;  // training inputs (rows x (D + 2)) and labels (rows)
  int64_t rows = 0, cap = 0;
  DevBuf gpart, gacc, chol, theta, flag;  // ridge mean
  DevBuf A0, Z[3], Hs[3], out, dz, dA, dB, perm, lossacc, xin;
  int64_t work_rows = 0;
  int64_t* perm_host = nullptr;
  int64_t perm_cap = 0;
  ~adasap_ws_s() {
    if (perm_host) (void)hipHostFree(perm_host);
  }
};

namespace {

constexpr int GT = 64;           // GEMM output tile
constexpr int GK = 16;           // GEMM depth stage
constexpr int CHUNK = 1 << 15;   // rows per streamed chunk
constexpr int GRAM_SPLITS = 16;  // row splits of one Gram chunk

enum { EPI_STORE = 0, EPI_BIAS_SILU = 1, EPI_DSILU = 2 };

__device__ inline float sigmoidf_(float z) {
  const float e = expf(-fabsf(z));
  return z >= 0.0f ? 1.0f / (1.0f + e) : e / (1.0f + e);
}

// ---------------------------------------------------------------- features and ridge mean

// A[i, j] = cos(x_i . omega_j + c_j) for j < D; A[i, D] = y_i
__global__ void cos_kernel(int64_t rows, int d, int D, const float* __restrict__ X,
                           const float* __restrict__ freqs, const float* __restrict__ phases,
                           const float* __restrict__ y, float* __restrict__ A, int64_t lda) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= rows * D) return;
  const int64_t i = e / D;
  const int j = (int)(e - i * D);
  const float* x = X + i * d;
  const float* w = freqs + (int64_t)j * d;
  float a = phases[j];
  for (int f = 0; f < d; ++f) a = fmaf(x[f], w[f], a);
  A[i * lda + j] = cosf(a);
  if (j == 0) A[i * lda + D] = y[i];
}

// partial Gram sums of the first C columns of F over one row split: lower tiles only
__global__ __launch_bounds__(256) void gram_kernel(int64_t rows, int C, const float* __restrict__ F,
                                                   int64_t ld, int64_t rps, double* __restrict__ part) {
  __shared__ float Fi[GK][GT + 1], Fj[GK][GT + 1];
  int ti = 0;
  const int p = blockIdx.x;
  while ((ti + 1) * (ti + 2) / 2 <= p) ++ti;
  const int tj = p - ti * (ti + 1) / 2;
  const int tid = threadIdx.x, tx = tid % 16, ty = tid / 16;
  double acc[4][4] = {};
  const int64_t r0 = (int64_t)blockIdx.y * rps;
  const int64_t r1 = r0 + rps < rows ? r0 + rps : rows;
  for (int64_t rb = r0; rb < r1; rb += GK) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = tid + 256 * q;
      const int rr = e / GT, cc = e % GT;
      const int64_t row = rb + rr;
      const int ci = ti * GT + cc, cj = tj * GT + cc;
      Fi[rr][cc] = (row < r1 && ci < C) ? F[row * ld + ci] : 0.0f;
      Fj[rr][cc] = (row < r1 && cj < C) ? F[row * ld + cj] : 0.0f;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < GK; ++k) {
      double a[4], b[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        a[u] = (double)Fi[k][ty * 4 + u];
        b[u] = (double)Fj[k][tx * 4 + u];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[u][v] = fma(a[u], b[v], acc[u][v]);
    }
    __syncthreads();
  }
  double* P = part + (int64_t)blockIdx.y * C * C;
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int gi = ti * GT + ty * 4 + u, gj = tj * GT + tx * 4 + v;
      if (gi < C && gj < C) P[(int64_t)gi * C + gj] = acc[u][v];
    }
}

// acc[e] += sum_s part[s][e] in split order, over the entries the lower tiles cover
__global__ void gram_reduce_kernel(int C, int splits, const double* __restrict__ part,
                                   double* __restrict__ acc) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)C * C) return;
  const int gi = (int)(e / C), gj = (int)(e % C);
  if (gi / GT < gj / GT) return;
  double s = acc[e];
  for (int q = 0; q < splits; ++q) s += part[(int64_t)q * C * C + e];
  acc[e] = s;
}

// theta = (Phi^T Phi + lam I)^{-1} Phi^T y from G = [cos | y]^T [cos | y] (C = D + 1):
// Phi^T Phi = (2/D) G[:D, :D], Phi^T y = sqrt(2/D) G[D, :D].  One workgroup; the lower
// triangle of L (D x D, float64) is factored in place by right-looking column steps.
__global__ __launch_bounds__(1024) void ridge_solve_kernel(int D, const double* __restrict__ G,
                                                           double lam, double* __restrict__ L,
                                                           double* __restrict__ theta,
                                                           int* __restrict__ flag) {
  __shared__ double bv[1024];
  const int tid = threadIdx.x, nt = blockDim.x;
  const int C = D + 1;
  const double sc = 2.0 / D, sq = sqrt(2.0 / D);
  for (int64_t e = tid; e < (int64_t)D * D; e += nt) {
    const int i = (int)(e / D), j = (int)(e % D);
    if (j <= i) L[e] = sc * G[(int64_t)i * C + j] + (i == j ? lam : 0.0);
  }
  for (int j = tid; j < D; j += nt) bv[j] = sq * G[(int64_t)D * C + j];
  __syncthreads();
  for (int j = 0; j < D; ++j) {
    if (tid == 0) {
      double dj = L[(int64_t)j * D + j];
      if (!(dj > 0.0)) {
        flag[0] = 1;
        dj = 1.0;
      }
      L[(int64_t)j * D + j] = sqrt(dj);
    }
    __syncthreads();
    const double ljj = L[(int64_t)j * D + j];
    for (int i = j + 1 + tid; i < D; i += nt) L[(int64_t)i * D + j] /= ljj;
    __syncthreads();
    const int w = D - j - 1;
    for (int64_t e = tid; e < (int64_t)w * w; e += nt) {
      const int ii = j + 1 + (int)(e / w), kk = j + 1 + (int)(e % w);
      if (kk <= ii) L[(int64_t)ii * D + kk] -= L[(int64_t)ii * D + j] * L[(int64_t)kk * D + j];
    }
    __syncthreads();
  }
  for (int j = 0; j < D; ++j) {  // L z = b
    if (tid == 0) bv[j] /= L[(int64_t)j * D + j];
    __syncthreads();
    for (int i = j + 1 + tid; i < D; i += nt) bv[i] -= L[(int64_t)i * D + j] * bv[j];
    __syncthreads();
  }
  for (int j = D - 1; j >= 0; --j) {  // L^T theta = z
    if (tid == 0) bv[j] /= L[(int64_t)j * D + j];
    __syncthreads();
    for (int i = tid; i < j; i += nt) bv[i] -= L[(int64_t)j * D + i] * bv[j];
    __syncthreads();
  }
  for (int j = tid; j < D; j += nt) theta[j] = bv[j];
}

// A[i, D + 1] = sqrt(2/D) sum_j A[i, j] theta_j (one wave per row, float64 sum)
__global__ __launch_bounds__(256) void mrff_kernel(int64_t rows, int D, float* __restrict__ A,
                                                   int64_t lda, const double* __restrict__ theta) {
  const int64_t i = (int64_t)blockIdx.x * 4 + threadIdx.x / 64;
  const int lane = threadIdx.x % 64;
  if (i >= rows) return;
  double s = 0.0;
  for (int j = lane; j < D; j += 64) s += (double)A[i * lda + j] * theta[j];
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  if (lane == 0) A[i * lda + D + 1] = (float)(sqrt(2.0 / D) * s);
}

// ---------------------------------------------------------------- dense layers

// C (M x N) = op(A) op(B): A is M x K (TA: stored K x M), B is K x N (TB: stored N x K).
// EPI_BIAS_SILU: z = acc + bias[n]; Z = z (if Z); C = silu(z).  EPI_DSILU: C = acc silu'(Z).
template <bool TA, bool TB, int EPI>
__global__ __launch_bounds__(256) void sgemm_kernel(int M, int N, int K, const float* __restrict__ A,
                                                    int64_t lda, const float* __restrict__ B,
                                                    int64_t ldb, float* __restrict__ C, int64_t ldc,
                                                    const float* __restrict__ bias,
                                                    float* __restrict__ Z, int64_t ldz) {
  __shared__ float As[GK][GT + 4], Bs[GK][GT + 4];
  const int tid = threadIdx.x, tx = tid % 16, ty = tid / 16;
  const int m0 = blockIdx.y * GT, n0 = blockIdx.x * GT;
  float acc[4][4] = {};
  for (int k0 = 0; k0 < K; k0 += GK) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = tid + 256 * q;
      int mi, ki;
      if (TA) {
        ki = e / GT;
        mi = e % GT;
      } else {
        mi = e / GK;
        ki = e % GK;
      }
      int gm = m0 + mi, gk = k0 + ki;
      As[ki][mi] = (gm < M && gk < K) ? (TA ? A[(int64_t)gk * lda + gm] : A[(int64_t)gm * lda + gk]) : 0.0f;
      int ni;
      if (TB) {
        ni = e / GK;
        ki = e % GK;
      } else {
        ki = e / GT;
        ni = e % GT;
      }
      const int gn = n0 + ni;
      gk = k0 + ki;
      Bs[ki][ni] = (gn < N && gk < K) ? (TB ? B[(int64_t)gn * ldb + gk] : B[(int64_t)gk * ldb + gn]) : 0.0f;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < GK; ++kk) {
      float a[4], b[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        a[u] = As[kk][ty * 4 + u];
        b[u] = Bs[kk][tx * 4 + u];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[u][v] = fmaf(a[u], b[v], acc[u][v]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int gm = m0 + ty * 4 + u;
    if (gm >= M) continue;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int gn = n0 + tx * 4 + v;
      if (gn >= N) continue;
      float r = acc[u][v];
      if (EPI == EPI_BIAS_SILU) {
        const float z = r + bias[gn];
        if (Z) Z[(int64_t)gm * ldz + gn] = z;
        r = z * sigmoidf_(z);
      } else if (EPI == EPI_DSILU) {
        const float z = Z[(int64_t)gm * ldz + gn];
        const float s = sigmoidf_(z);
        r *= s * (1.0f + z * (1.0f - s));
      }
      C[(int64_t)gm * ldc + gn] = r;
    }
  }
}

// out[i] = H[i, :] . w + b (one wave per row)
__global__ __launch_bounds__(256) void out_layer_kernel(int64_t rows, int Hd, const float* __restrict__ H,
                                                        const float* __restrict__ w,
                                                        const float* __restrict__ b,
                                                        float* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * 4 + threadIdx.x / 64;
  const int lane = threadIdx.x % 64;
  if (i >= rows) return;
  float s = 0.0f;
  for (int k = lane; k < Hd; k += 64) s = fmaf(H[i * Hd + k], w[k], s);
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  if (lane == 0) out[i] = s + b[0];
}

// dz = (2/m)(out - t); lossacc[0] += sum (out - t)^2; lossacc[1] = that sum / m (one block)
__global__ __launch_bounds__(256) void loss_kernel(int m, const float* __restrict__ out,
                                                   const float* __restrict__ t, float* __restrict__ dz,
                                                   double* __restrict__ lossacc) {
  __shared__ double red[256];
  double s = 0.0;
  for (int i = threadIdx.x; i < m; i += 256) {
    const float r = out[i] - t[i];
    dz[i] = (2.0f / (float)m) * r;
    s += (double)r * (double)r;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    lossacc[0] += red[0];
    lossacc[1] = red[0] / m;
  }
}

// output layer backward: dZ3[i, k] = dz_i w_k silu'(Z3[i, k])
__global__ void last_back_kernel(int64_t m, int Hd, const float* __restrict__ dz,
                                 const float* __restrict__ w, const float* __restrict__ Z3,
                                 float* __restrict__ dZ3) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= m * Hd) return;
  const int64_t i = e / Hd;
  const int k = (int)(e - i * Hd);
  const float z = Z3[e];
  const float s = sigmoidf_(z);
  dZ3[e] = dz[i] * w[k] * (s * (1.0f + z * (1.0f - s)));
}

// out[c] = sum_i X[i, c] (W: times wt[i] if wt) for c < N; 256 threads per 64 columns,
// four row groups combined in a fixed order
__global__ __launch_bounds__(256) void colsum_kernel(int64_t m, int N, const float* __restrict__ X,
                                                     int64_t ld, const float* __restrict__ wt,
                                                     float* __restrict__ out) {
  __shared__ float red[4][64];
  const int c = blockIdx.x * 64 + threadIdx.x % 64;
  const int g = threadIdx.x / 64;
  float s = 0.0f;
  if (c < N)
    for (int64_t i = g; i < m; i += 4) s += wt ? X[i * ld + c] * wt[i] : X[i * ld + c];
  red[g][threadIdx.x % 64] = s;
  __syncthreads();
  if (g == 0 && c < N) out[c] = (red[0][threadIdx.x] + red[1][threadIdx.x]) + (red[2][threadIdx.x] + red[3][threadIdx.x]);
}

__global__ void sum_kernel(int64_t m, const float* __restrict__ x, float* __restrict__ out) {
  __shared__ float red[256];
  float s = 0.0f;
  for (int64_t i = threadIdx.x; i < m; i += 256) s += x[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = red[0];
}

__global__ void adam_kernel(int64_t np, float* __restrict__ p, const float* __restrict__ g,
                            float* __restrict__ mo, float* __restrict__ vo, float lr, float b1,
                            float b2, float eps, float c1, float c2) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= np) return;
  const float gi = g[e];
  const float m = b1 * mo[e] + (1.0f - b1) * gi;
  const float v = b2 * vo[e] + (1.0f - b2) * gi * gi;
  mo[e] = m;
  vo[e] = v;
  p[e] -= lr * (m * c1) / (sqrtf(v * c2) + eps);
}

__global__ void gather_kernel(int64_t rows, int cols, const float* __restrict__ src, int64_t lds,
                              const int64_t* __restrict__ idx, float* __restrict__ dst,
                              const float* __restrict__ tsrc, float* __restrict__ tdst) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= rows * cols) return;
  const int64_t i = e / cols;
  const int c = (int)(e - i * cols);
  const int64_t r = idx[i];
  dst[i * cols + c] = src[r * lds + c];
  if (c == 0) tdst[i] = tsrc[r];
}

// t = y - lam W (labels) or W0 = (y - mhat) / lam (initial iterate)
__global__ void axpby_kernel(int64_t n, const float* __restrict__ y, const float* __restrict__ z,
                             double a, double c, float* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = (float)(((double)y[i] + a * (double)z[i]) * c);
}

__global__ void flag_zero_kernel(int* f) { f[0] = 0; }

unsigned blocks_for(int64_t n, int t = 256) { return (unsigned)((n + t - 1) / t); }

adasap_status_t ws_invalid(const char* m) {
  set_error(m);
  return ADASAP_ERR_INVALID_ARG;
}

bool cfg_ok(const adasap_ws_config_t* c) {
  return c && c->struct_size == sizeof(adasap_ws_config_t) && c->d >= 1 && c->d <= 64 &&
         c->D >= 1 && c->D <= 1024 && c->hidden >= 1 && c->hidden <= 1024 &&
         std::isfinite(c->lambda) && c->lambda > 0 && c->beta1 >= 0 && c->beta1 < 1 &&
         c->beta2 >= 0 && c->beta2 < 1 && c->adam_eps >= 0;
}

int64_t count_params(const adasap_ws_config_t* c, int64_t* offW, int64_t* offB) {
  const int64_t sizes[5] = {c->D + 2, c->hidden, c->hidden, c->hidden, 1};
  int64_t off = 0;
  for (int l = 0; l < 4; ++l) {
    if (offW) offW[l] = off;
    off += sizes[l + 1] * sizes[l];
    if (offB) offB[l] = off;
    off += sizes[l + 1];
  }
  return off;
}

adasap_status_t ensure_work(adasap_ws_t ws, int64_t rows) {
  if (rows <= ws->work_rows) return ADASAP_OK;
  const int64_t Hd = ws->cfg.hidden, C2 = ws->cfg.D + 2;
  ADASAP_TRY(ws->A0.ensure((size_t)rows * C2 * 4));
  for (int l = 0; l < 3; ++l) {
    ADASAP_TRY(ws->Z[l].ensure((size_t)rows * Hd * 4));
    ADASAP_TRY(ws->Hs[l].ensure((size_t)rows * Hd * 4));
  }
  ADASAP_TRY(ws->out.ensure((size_t)rows * 4));
  ADASAP_TRY(ws->dz.ensure((size_t)rows * 4));
  ADASAP_TRY(ws->xin.ensure((size_t)rows * 4));
  ADASAP_TRY(ws->dA.ensure((size_t)rows * Hd * 4));
  ADASAP_TRY(ws->dB.ensure((size_t)rows * Hd * 4));
  ws->work_rows = rows;
  return ADASAP_OK;
}

template <bool TA, bool TB, int EPI>
adasap_status_t gemm(int M, int N, int K, const float* A, int64_t lda, const float* B, int64_t ldb,
                     float* C, int64_t ldc, const float* bias, float* Z, int64_t ldz, hipStream_t s) {
  if (M <= 0 || N <= 0) return ADASAP_OK;
  dim3 grid((unsigned)((N + GT - 1) / GT), (unsigned)((M + GT - 1) / GT));
  hipLaunchKernelGGL((sgemm_kernel<TA, TB, EPI>), grid, dim3(256), 0, s, M, N, K, A, lda, B, ldb,
                     C, ldc, bias, Z, ldz);
  ADASAP_LAUNCH_CHECK();
  return ADASAP_OK;
}

// forward pass of `rows` input rows A (ld D + 2); keep_z stores the pre-activations
adasap_status_t forward(adasap_ws_t ws, int64_t rows, const float* A, bool keep_z) {
  const int Hd = ws->cfg.hidden, C2 = ws->cfg.D + 2;
  const float* P = ws->params.as<float>();
  hipStream_t s = ws->s;
  const float* in = A;
  int64_t ldin = C2;
  int kin = C2;
  for (int l = 0; l < 3; ++l) {
    ADASAP_TRY((gemm<false, true, EPI_BIAS_SILU>((int)rows, Hd, kin, in, ldin, P + ws->offW[l], kin,
                                                 ws->Hs[l].as<float>(), Hd, P + ws->offB[l],
                                                 keep_z ? ws->Z[l].as<float>() : nullptr, Hd, s)));
    in = ws->Hs[l].as<float>();
    ldin = Hd;
    kin = Hd;
  }
  hipLaunchKernelGGL(out_layer_kernel, dim3(blocks_for(rows, 4)), dim3(256), 0, s, rows, Hd,
                     ws->Hs[2].as<float>(), P + ws->offW[3], P + ws->offB[3], ws->out.as<float>());
  ADASAP_LAUNCH_CHECK();
  return ADASAP_OK;
}

// loss and gradient (into ws->grad) for `m` rows A with labels t
adasap_status_t loss_grad(adasap_ws_t ws, int64_t m, const float* A, const float* t) {
  const int Hd = ws->cfg.hidden, C2 = ws->cfg.D + 2;
  const float* P = ws->params.as<float>();
  float* G = ws->grad.as<float>();
  hipStream_t s = ws->s;
  ADASAP_TRY(forward(ws, m, A, true));
  hipLaunchKernelGGL(loss_kernel, dim3(1), dim3(256), 0, s, (int)m, ws->out.as<float>(), t,
                     ws->dz.as<float>(), ws->lossacc.as<double>());
  ADASAP_LAUNCH_CHECK();
  // output layer: dW4 = dz^T H3, db4 = sum dz, dZ3 = dz w4^T o silu'(Z3)
  hipLaunchKernelGGL(colsum_kernel, dim3(blocks_for(Hd, 64)), dim3(256), 0, s, m, Hd,
                     ws->Hs[2].as<float>(), (int64_t)Hd, ws->dz.as<float>(), G + ws->offW[3]);
  ADASAP_LAUNCH_CHECK();
  hipLaunchKernelGGL(sum_kernel, dim3(1), dim3(256), 0, s, m, ws->dz.as<float>(), G + ws->offB[3]);
  ADASAP_LAUNCH_CHECK();
  hipLaunchKernelGGL(last_back_kernel, dim3(blocks_for(m * Hd)), dim3(256), 0, s, m, Hd,
                     ws->dz.as<float>(), P + ws->offW[3], ws->Z[2].as<float>(), ws->dA.as<float>());
  ADASAP_LAUNCH_CHECK();
  float* dcur = ws->dA.as<float>();
  float* dnext = ws->dB.as<float>();
  for (int l = 2; l >= 0; --l) {
    const float* prev = l > 0 ? ws->Hs[l - 1].as<float>() : A;
    const int kin = l > 0 ? Hd : C2;
    // dW_l = dZ_l^T prev (Hd x kin), db_l = colsum dZ_l
    ADASAP_TRY((gemm<true, false, EPI_STORE>(Hd, kin, (int)m, dcur, Hd, prev, kin, G + ws->offW[l], kin,
                                             nullptr, nullptr, 0, s)));
    hipLaunchKernelGGL(colsum_kernel, dim3(blocks_for(Hd, 64)), dim3(256), 0, s, m, Hd, dcur,
                       (int64_t)Hd, nullptr, G + ws->offB[l]);
    ADASAP_LAUNCH_CHECK();
    if (l > 0) {
      // dZ_{l-1} = (dZ_l W_l) o silu'(Z_{l-1})
      ADASAP_TRY((gemm<false, false, EPI_DSILU>((int)m, Hd, Hd, dcur, Hd, P + ws->offW[l], Hd, dnext, Hd,
                                                nullptr, ws->Z[l - 1].as<float>(), Hd, s)));
      float* tmp = dcur;
      dcur = dnext;
      dnext = tmp;
    }
  }
  return ADASAP_OK;
}

// ridge weights over n points: Gram of [cos | y] accumulated chunk by chunk, then solved
adasap_status_t ridge(adasap_ws_t ws, int64_t n, const float* X, const float* y, float* Amat) {
  const int D = ws->cfg.D, d = ws->cfg.d, C = D + 1, C2 = D + 2;
  hipStream_t s = ws->s;
  ADASAP_TRY(ws->gacc.ensure((size_t)C * C * 8));
  ADASAP_TRY(ws->gpart.ensure((size_t)GRAM_SPLITS * C * C * 8));
  ADASAP_TRY(ws->chol.ensure((size_t)D * D * 8));
  ADASAP_TRY(ws->theta.ensure((size_t)D * 8));
  ADASAP_TRY(ws->flag.ensure(sizeof(int)));
  ADASAP_HIP(hipMemsetAsync(ws->gacc.p, 0, (size_t)C * C * 8, s));
  hipLaunchKernelGGL(flag_zero_kernel, dim3(1), dim3(1), 0, s, ws->flag.as<int>());
  ADASAP_LAUNCH_CHECK();
  const int T = (C + GT - 1) / GT;
  for (int64_t i0 = 0; i0 < n; i0 += CHUNK) {
    const int64_t rows = n - i0 < CHUNK ? n - i0 : CHUNK;
    if (!Amat) ADASAP_TRY(ensure_work(ws, rows));
    float* F = Amat ? Amat + i0 * C2 : ws->A0.as<float>();
    hipLaunchKernelGGL(cos_kernel, dim3(blocks_for(rows * D)), dim3(256), 0, s, rows, d, D,
                       X + i0 * d, ws->freqs.as<float>(), ws->phases.as<float>(), y + i0, F,
                       (int64_t)C2);
    ADASAP_LAUNCH_CHECK();
    const int64_t rps = ((rows + GRAM_SPLITS - 1) / GRAM_SPLITS + GK - 1) / GK * GK;
    const int splits = (int)((rows + rps - 1) / rps);
    hipLaunchKernelGGL(gram_kernel, dim3((unsigned)(T * (T + 1) / 2), (unsigned)splits), dim3(256), 0, s,
                       rows, C, F, (int64_t)C2, rps, ws->gpart.as<double>());
    ADASAP_LAUNCH_CHECK();
    hipLaunchKernelGGL(gram_reduce_kernel, dim3(blocks_for((int64_t)C * C)), dim3(256), 0, s, C, splits,
                       ws->gpart.as<double>(), ws->gacc.as<double>());
    ADASAP_LAUNCH_CHECK();
  }
  hipLaunchKernelGGL(ridge_solve_kernel, dim3(1), dim3(1024), 0, s, D, ws->gacc.as<double>(),
                     ws->cfg.lambda, ws->chol.as<double>(), ws->theta.as<double>(), ws->flag.as<int>());
  ADASAP_LAUNCH_CHECK();
  int hf = 0;
  ADASAP_HIP(hipMemcpyAsync(&hf, ws->flag.p, sizeof(int), hipMemcpyDeviceToHost, s));
  ADASAP_HIP(hipStreamSynchronize(s));
  if (hf) {
    set_error("ridge system of the Fourier features is not positive definite");
    return ADASAP_ERR_NOT_PD;
  }
  return ADASAP_OK;
}

// network inputs of rows [i0, i0 + rows) into F (ld D + 2), with the ridge weights in ws->theta
adasap_status_t inputs_chunk(adasap_ws_t ws, int64_t rows, const float* X, const float* y, float* F,
                             bool have_cos) {
  const int D = ws->cfg.D, d = ws->cfg.d, C2 = D + 2;
  hipStream_t s = ws->s;
  if (!have_cos) {
    hipLaunchKernelGGL(cos_kernel, dim3(blocks_for(rows * D)), dim3(256), 0, s, rows, d, D, X,
                       ws->freqs.as<float>(), ws->phases.as<float>(), y, F, (int64_t)C2);
    ADASAP_LAUNCH_CHECK();
  }
  hipLaunchKernelGGL(mrff_kernel, dim3(blocks_for(rows, 4)), dim3(256), 0, s, rows, D, F, (int64_t)C2,
                     ws->theta.as<double>());
  ADASAP_LAUNCH_CHECK();
  return ADASAP_OK;
}

adasap_status_t check_points(adasap_ws_t ws, int64_t n, const float* X, const float* y) {
  if (!ws) return ws_invalid("warm-start object is null");
  if (n < 1) return ws_invalid("n must be >= 1");
  if (!X || !y) return ws_invalid("X and y must be non-null device pointers");
  return ADASAP_OK;
}

// predicted mean of n points into mhat (float32), chunk by chunk
adasap_status_t predict(adasap_ws_t ws, int64_t n, const float* X, const float* y, float* mhat) {
  ADASAP_TRY(ridge(ws, n, X, y, nullptr));
  const int d = ws->cfg.d;
  for (int64_t i0 = 0; i0 < n; i0 += CHUNK) {
    const int64_t rows = n - i0 < CHUNK ? n - i0 : CHUNK;
    ADASAP_TRY(ensure_work(ws, rows));
    ADASAP_TRY(inputs_chunk(ws, rows, X + i0 * d, y + i0, ws->A0.as<float>(), false));
    ADASAP_TRY(forward(ws, rows, ws->A0.as<float>(), false));
    ADASAP_HIP(hipMemcpyAsync(mhat + i0, ws->out.p, rows * 4, hipMemcpyDeviceToDevice, ws->s));
  }
  return ADASAP_OK;
}

}  // namespace

extern "C" {

adasap_status_t adasap_ws_config_default(adasap_ws_config_t* cfg) {
  if (!cfg) return ws_invalid("cfg is null");
  std::memset(cfg, 0, sizeof(*cfg));
  cfg->struct_size = sizeof(adasap_ws_config_t);
  cfg->d = 9;
  cfg->D = 512;
  cfg->hidden = 256;
  cfg->lambda = 1e-2;
  cfg->beta1 = 0.9;
  cfg->beta2 = 0.999;
  cfg->adam_eps = 1e-8;
  return ADASAP_OK;
}

int64_t adasap_ws_param_count(const adasap_ws_config_t* cfg) {
  if (!cfg_ok(cfg)) return 0;
  return count_params(cfg, nullptr, nullptr);
}

adasap_status_t adasap_ws_create(const adasap_ws_config_t* cfg, const float* freqs,
                                 const float* phases, const float* params, void* stream,
                                 adasap_ws_t* out) {
  if (!out) return ws_invalid("out pointer is null");
  *out = nullptr;
  if (!cfg_ok(cfg)) return ws_invalid("invalid warm-start config (struct_size, d, D, hidden, lambda or Adam constants)");
  if (!freqs || !phases || !params) return ws_invalid("freqs, phases and params must be non-null device pointers");
  auto* ws = new (std::nothrow) adasap_ws_s();
  if (!ws) return ADASAP_ERR_OOM;
  ws->cfg = *cfg;
  ws->s = static_cast<hipStream_t>(stream);
  ws->np = count_params(cfg, ws->offW, ws->offB);
  auto fail = [&](adasap_status_t st) {
    delete ws;
    return st;
  };
  adasap_status_t st;
  const size_t pb = (size_t)ws->np * 4;
  if ((st = ws->freqs.ensure((size_t)cfg->D * cfg->d * 4)) != ADASAP_OK ||
      (st = ws->phases.ensure((size_t)cfg->D * 4)) != ADASAP_OK ||
      (st = ws->params.ensure(pb)) != ADASAP_OK || (st = ws->grad.ensure(pb)) != ADASAP_OK ||
      (st = ws->adam_m.ensure(pb)) != ADASAP_OK || (st = ws->adam_v.ensure(pb)) != ADASAP_OK ||
      (st = ws->lossacc.ensure(2 * sizeof(double))) != ADASAP_OK)
    return fail(st);
  if (hipMemcpyAsync(ws->freqs.p, freqs, (size_t)cfg->D * cfg->d * 4, hipMemcpyDeviceToDevice, ws->s) != hipSuccess ||
      hipMemcpyAsync(ws->phases.p, phases, (size_t)cfg->D * 4, hipMemcpyDeviceToDevice, ws->s) != hipSuccess ||
      hipMemcpyAsync(ws->params.p, params, pb, hipMemcpyDeviceToDevice, ws->s) != hipSuccess ||
      hipMemsetAsync(ws->adam_m.p, 0, pb, ws->s) != hipSuccess ||
      hipMemsetAsync(ws->adam_v.p, 0, pb, ws->s) != hipSuccess ||
      hipStreamSynchronize(ws->s) != hipSuccess) {
    set_error("device copy failed in adasap_ws_create");
    return fail(ADASAP_ERR_DEVICE);
  }
  *out = ws;
  return ADASAP_OK;
}

adasap_status_t adasap_ws_add_problem(adasap_ws_t ws, int64_t n, const float* X, const float* y,
                                      const float* W) {
  ADASAP_TRY(check_points(ws, n, X, y));
  if (!W) return ws_invalid("W must be a non-null device pointer");
  const int C2 = ws->cfg.D + 2;
  const int64_t need = ws->rows + n;
  if (need > ws->cap) {
    int64_t cap = ws->cap > 0 ? ws->cap : 1 << 16;
    while (cap < need) cap *= 2;
    DevBuf nA, nt;
    ADASAP_TRY(nA.ensure((size_t)cap * C2 * 4));
    ADASAP_TRY(nt.ensure((size_t)cap * 4));
    if (ws->rows > 0) {
      ADASAP_HIP(hipMemcpyAsync(nA.p, ws->trainA.p, (size_t)ws->rows * C2 * 4, hipMemcpyDeviceToDevice, ws->s));
      ADASAP_HIP(hipMemcpyAsync(nt.p, ws->traint.p, (size_t)ws->rows * 4, hipMemcpyDeviceToDevice, ws->s));
      ADASAP_HIP(hipStreamSynchronize(ws->s));
    }
    std::swap(ws->trainA.p, nA.p);
    std::swap(ws->trainA.bytes, nA.bytes);
    std::swap(ws->traint.p, nt.p);
    std::swap(ws->traint.bytes, nt.bytes);
    ws->cap = cap;
  }
  float* F = ws->trainA.as<float>() + ws->rows * C2;
  ADASAP_TRY(ridge(ws, n, X, y, F));
  ADASAP_TRY(inputs_chunk(ws, n, X, y, F, true));
  hipLaunchKernelGGL(axpby_kernel, dim3(blocks_for(n)), dim3(256), 0, ws->s, n, y, W, -ws->cfg.lambda, 1.0,
                     ws->traint.as<float>() + ws->rows);
  ADASAP_LAUNCH_CHECK();
  ADASAP_HIP(hipStreamSynchronize(ws->s));
  ws->rows = need;
  return ADASAP_OK;
}

int64_t adasap_ws_train_rows(adasap_ws_t ws) { return ws ? ws->rows : 0; }

adasap_status_t adasap_ws_train(adasap_ws_t ws, int32_t epochs, int32_t batch, double lr,
                                uint64_t seed, double* epoch_loss) {
  if (!ws) return ws_invalid("warm-start object is null");
  if (epochs < 0 || batch < 1 || batch > (1 << 16)) return ws_invalid("need epochs >= 0 and 1 <= batch <= 65536");
  if (!(lr > 0) || !std::isfinite(lr)) return ws_invalid("lr must be finite and > 0");
  if (ws->rows < 1) return ws_invalid("the training set is empty");
  const int64_t m = ws->rows;
  const int C2 = ws->cfg.D + 2;
  hipStream_t s = ws->s;
  ADASAP_TRY(ensure_work(ws, batch));
  ADASAP_TRY(ws->perm.ensure((size_t)m * 8));
  if (ws->perm_cap < m) {
    if (ws->perm_host) (void)hipHostFree(ws->perm_host);
    ws->perm_host = nullptr;
    ADASAP_HIP(hipHostMalloc((void**)&ws->perm_host, (size_t)m * 8));
    ws->perm_cap = m;
  }
  DevBuf bt;
  ADASAP_TRY(bt.ensure((size_t)batch * 4));
  for (int e = 0; e < epochs; ++e) {
    ADASAP_HIP(hipStreamSynchronize(s));  // the pinned order buffer is free
    permutation_host(seed, PURPOSE_MINIBATCH, (uint64_t)e, m, ws->perm_host);
    ADASAP_HIP(hipMemcpyAsync(ws->perm.p, ws->perm_host, (size_t)m * 8, hipMemcpyHostToDevice, s));
    ADASAP_HIP(hipMemsetAsync(ws->lossacc.p, 0, 2 * sizeof(double), s));
    for (int64_t i0 = 0; i0 < m; i0 += batch) {
      const int64_t rows = m - i0 < batch ? m - i0 : batch;
      hipLaunchKernelGGL(gather_kernel, dim3(blocks_for(rows * C2)), dim3(256), 0, s, rows, C2,
                         ws->trainA.as<float>(), (int64_t)C2, ws->perm.as<int64_t>() + i0,
                         ws->A0.as<float>(), ws->traint.as<float>(), bt.as<float>());
      ADASAP_LAUNCH_CHECK();
      ADASAP_TRY(loss_grad(ws, rows, ws->A0.as<float>(), bt.as<float>()));
      ++ws->adam_t;
      const double c1 = 1.0 / (1.0 - std::pow(ws->cfg.beta1, (double)ws->adam_t));
      const double c2 = 1.0 / (1.0 - std::pow(ws->cfg.beta2, (double)ws->adam_t));
      hipLaunchKernelGGL(adam_kernel, dim3(blocks_for(ws->np)), dim3(256), 0, s, ws->np,
                         ws->params.as<float>(), ws->grad.as<float>(), ws->adam_m.as<float>(),
                         ws->adam_v.as<float>(), (float)lr, (float)ws->cfg.beta1, (float)ws->cfg.beta2,
                         (float)ws->cfg.adam_eps, (float)c1, (float)c2);
      ADASAP_LAUNCH_CHECK();
    }
    double la[2];
    ADASAP_HIP(hipMemcpyAsync(la, ws->lossacc.p, sizeof(la), hipMemcpyDeviceToHost, s));
    ADASAP_HIP(hipStreamSynchronize(s));
    if (epoch_loss) epoch_loss[e] = la[0] / (double)m;
  }
  ADASAP_HIP(hipStreamSynchronize(s));
  return ADASAP_OK;
}

adasap_status_t adasap_ws_features(adasap_ws_t ws, int64_t n, const float* X, const float* y,
                                   float* out, double* theta) {
  ADASAP_TRY(check_points(ws, n, X, y));
  if (!out) return ws_invalid("out must be a non-null device pointer");
  ADASAP_TRY(ridge(ws, n, X, y, out));
  ADASAP_TRY(inputs_chunk(ws, n, X, y, out, true));
  if (theta)
    ADASAP_HIP(hipMemcpyAsync(theta, ws->theta.p, (size_t)ws->cfg.D * 8, hipMemcpyDeviceToDevice, ws->s));
  ADASAP_HIP(hipStreamSynchronize(ws->s));
  return ADASAP_OK;
}

adasap_status_t adasap_ws_loss_grad(adasap_ws_t ws, int64_t m, const float* A, const float* t,
                                    double* loss, float* grad) {
  if (!ws) return ws_invalid("warm-start object is null");
  if (m < 1 || m > (1 << 16)) return ws_invalid("need 1 <= m <= 65536");
  if (!A || !t || !grad) return ws_invalid("A, t and grad must be non-null device pointers");
  ADASAP_TRY(ensure_work(ws, m));
  ADASAP_HIP(hipMemsetAsync(ws->lossacc.p, 0, 2 * sizeof(double), ws->s));
  ADASAP_TRY(loss_grad(ws, m, A, t));
  ADASAP_HIP(hipMemcpyAsync(grad, ws->grad.p, (size_t)ws->np * 4, hipMemcpyDeviceToDevice, ws->s));
  double la[2];
  ADASAP_HIP(hipMemcpyAsync(la, ws->lossacc.p, sizeof(la), hipMemcpyDeviceToHost, ws->s));
  ADASAP_HIP(hipStreamSynchronize(ws->s));
  if (loss) *loss = la[1];
  return ADASAP_OK;
}

adasap_status_t adasap_ws_predict_mean(adasap_ws_t ws, int64_t n, const float* X, const float* y,
                                       float* mhat) {
  ADASAP_TRY(check_points(ws, n, X, y));
  if (!mhat) return ws_invalid("mhat must be a non-null device pointer");
  ADASAP_TRY(predict(ws, n, X, y, mhat));
  ADASAP_HIP(hipStreamSynchronize(ws->s));
  return ADASAP_OK;
}

adasap_status_t adasap_ws_initial_iterate(adasap_ws_t ws, int64_t n, const float* X,
                                          const float* y, float* W0) {
  ADASAP_TRY(check_points(ws, n, X, y));
  if (!W0) return ws_invalid("W0 must be a non-null device pointer");
  ADASAP_TRY(predict(ws, n, X, y, W0));
  hipLaunchKernelGGL(axpby_kernel, dim3(blocks_for(n)), dim3(256), 0, ws->s, n, y, W0, -1.0,
                     1.0 / ws->cfg.lambda, W0);
  ADASAP_LAUNCH_CHECK();
  ADASAP_HIP(hipStreamSynchronize(ws->s));
  return ADASAP_OK;
}

adasap_status_t adasap_ws_get_params(adasap_ws_t ws, float* out) {
  if (!ws || !out) return ws_invalid("null argument");
  ADASAP_HIP(hipMemcpyAsync(out, ws->params.p, (size_t)ws->np * 4, hipMemcpyDeviceToDevice, ws->s));
  ADASAP_HIP(hipStreamSynchronize(ws->s));
  return ADASAP_OK;
}

adasap_status_t adasap_ws_set_params(adasap_ws_t ws, const float* in) {
  if (!ws || !in) return ws_invalid("null argument");
  ADASAP_HIP(hipMemcpyAsync(ws->params.p, in, (size_t)ws->np * 4, hipMemcpyDeviceToDevice, ws->s));
  ADASAP_HIP(hipStreamSynchronize(ws->s));
  return ADASAP_OK;
}

void adasap_ws_destroy(adasap_ws_t ws) {
  if (ws) {
    (void)hipStreamSynchronize(ws->s);
    delete ws;
  }
}

}  // extern "C"
