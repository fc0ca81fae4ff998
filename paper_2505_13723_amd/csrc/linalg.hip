// Float64 dense linear algebra of Step III/IV (Appendix, "Randomized Nystrom
// approximation" and "Computing the stepsize"): Gram products, small GEMMs, the
// one-workgroup Cholesky of the Nystrom core with its triangular inverse, a cyclic
// Jacobi eigensolver for the r x r Gram matrix of B = Y_nu R^{-1}, the sorting/shift
// removal of Alg. NysApprox and the vector reductions of randomized powering.
// r <= 128 throughout, so every r x r matrix fits one workgroup's LDS (160 KB on gfx950).
#include "internal.h"

namespace adasap {

namespace {

constexpr int RMAX = 128;

__device__ inline double ld_any(const void* p, DT t, int64_t i) {
  return t == DT::F64 ? static_cast<const double*>(p)[i] : (double)static_cast<const float*>(p)[i];
}

// p advanced by e elements of type t
__device__ inline const void* adv(const void* p, DT t, int64_t e) {
  return static_cast<const char*>(p) + e * (t == DT::F64 ? 8 : 4);
}

// ---------------------------------------------------------------- Gram products P = A^T B
constexpr int G_T = 64;     // output tile of the Gram kernel (4 x 4 entries per thread)
constexpr int G_ROWS = 16;  // rows staged per step

// The small dense kernels of the Nystrom factors and of powering run on a second stream
// beside the long kernel-block product; a raised wave priority lets their (few) waves win
// instruction issue on the SIMDs they share with it.
__device__ inline void raise_wave_priority() { __builtin_amdgcn_s_setprio(2); }

// A^T B over a row range: a 64 x 64 output tile per workgroup, 4 x 4 entries per thread
// (entries ty + 16 i, tx + 16 j, so the LDS reads of a wave are conflict-free), 16 rows
// staged per barrier; blockIdx.z = problem * nsplit + row split.
__global__ __launch_bounds__(256) void gram_partial_kernel(int64_t rows, int p, int q,
                                                           const void* __restrict__ A, DT at,
                                                           int64_t lda, const void* __restrict__ B,
                                                           DT bt, int64_t ldb,
                                                           double* __restrict__ part, int nsplit,
                                                           int64_t chunk, Batch bat) {
  raise_wave_priority();
  __shared__ double As[G_ROWS][G_T];
  __shared__ double Bs[G_ROWS][G_T];
  const int prob = blockIdx.z / nsplit, split = blockIdx.z % nsplit;
  A = adv(A, at, prob * bat.sA);
  B = adv(B, bt, prob * bat.sB);
  part += (int64_t)prob * nsplit * p * q;
  const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
  const int p0 = blockIdx.y * G_T, q0 = blockIdx.x * G_T;
  const int64_t r0 = (int64_t)split * chunk;
  const int64_t r1 = r0 + chunk < rows ? r0 + chunk : rows;
  double acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = 0.0;
  for (int64_t rr = r0; rr < r1; rr += G_ROWS) {
#pragma unroll
    for (int u = 0; u < (G_ROWS * G_T) / 256; ++u) {
      const int e = threadIdx.x + u * 256;
      const int lr = e / G_T, lc = e % G_T;
      const int64_t row = rr + lr;
      As[lr][lc] = (row < r1 && p0 + lc < p) ? ld_any(A, at, row * lda + p0 + lc) : 0.0;
      Bs[lr][lc] = (row < r1 && q0 + lc < q) ? ld_any(B, bt, row * ldb + q0 + lc) : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int l = 0; l < G_ROWS; ++l) {
      double av[4], bv[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) av[i] = As[l][ty + 16 * i];
#pragma unroll
      for (int j = 0; j < 4; ++j) bv[j] = Bs[l][tx + 16 * j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] += av[i] * bv[j];
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int pi = p0 + ty + 16 * i;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int qj = q0 + tx + 16 * j;
      if (pi < p && qj < q) part[((int64_t)split * p + pi) * q + qj] = acc[i][j];
    }
  }
}

__global__ void gram_reduce_kernel(const double* __restrict__ part, int splits, int p, int q,
                                   const double* __restrict__ rowscale, double* __restrict__ P,
                                   Batch bat) {
  raise_wave_priority();
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= p * q) return;
  const int prob = blockIdx.y;
  part += (int64_t)prob * splits * p * q;
  P += prob * bat.sC;
  if (rowscale) rowscale += prob * bat.sD;
  double s = 0.0;
  // (the loads of eight splits are issued together; the sum keeps the split order)
#pragma unroll 8
  for (int sp = 0; sp < splits; ++sp) s += part[(int64_t)sp * p * q + e];
  if (rowscale) s *= rowscale[e / q];
  P[e] = s;
}

// The same sum over many partials: one block per output entry, a strided sum per thread
// and a fixed-order tree.
__global__ __launch_bounds__(256) void gram_reduce_tree_kernel(const double* __restrict__ part,
                                                               int splits, int p, int q,
                                                               const double* __restrict__ rowscale,
                                                               double* __restrict__ P, Batch bat) {
  raise_wave_priority();
  __shared__ double red[256];
  const int e = blockIdx.x;
  const int prob = blockIdx.y;
  part += (int64_t)prob * splits * p * q;
  P += prob * bat.sC;
  if (rowscale) rowscale += prob * bat.sD;
  double s = 0.0;
  for (int sp = threadIdx.x; sp < splits; sp += 256) s += part[(int64_t)sp * p * q + e];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) P[e] = rowscale ? red[0] * rowscale[e / q] : red[0];
}

// Gram products with a thin right factor (q <= 4): one thread per column of A, rows in
// two interleaved halves, so every load of a row of A is coalesced.  Row chunks are sized
// so that a launch has about 256 workgroups (at least 64 rows each).
__global__ __launch_bounds__(256) void gramv_partial_kernel(int64_t rows, int p, int q,
                                                            const void* __restrict__ A, DT at,
                                                            int64_t lda, const void* __restrict__ B,
                                                            DT bt, int64_t ldb,
                                                            double* __restrict__ part, Batch bat,
                                                            int64_t chunk) {
  raise_wave_priority();
  __shared__ double red[128 * 4];
  const int prob = blockIdx.y;
  A = adv(A, at, prob * bat.sA);
  B = adv(B, bt, prob * bat.sB);
  part += (int64_t)prob * gridDim.x * p * q;
  const int col = threadIdx.x % 128, half = threadIdx.x / 128;
  const int64_t r0 = (int64_t)blockIdx.x * chunk;
  const int64_t r1 = r0 + chunk < rows ? r0 + chunk : rows;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  if (col < p) {
    for (int64_t row = r0 + half; row < r1; row += 2) {
      const double a = ld_any(A, at, row * lda + col);
#pragma unroll
      for (int c = 0; c < 4; ++c)
        if (c < q) acc[c] += a * ld_any(B, bt, row * ldb + c);
    }
  }
  if (half == 1)
    for (int c = 0; c < 4; ++c) red[col * 4 + c] = acc[c];
  __syncthreads();
  if (half == 0 && col < p)
    for (int c = 0; c < q; ++c) part[((int64_t)blockIdx.x * p + col) * q + c] = acc[c] + red[col * 4 + c];
}

// OUT = f E + A M for a thin M (q <= 4): 32 rows of A (p <= 128 entries) per workgroup, 8 per
// wave with their loads in flight together (M staged in LDS once per workgroup)
// (QM: the largest q of the instantiation; q = 1, the powering and single right-hand-side
// directions, keeps 8 accumulators instead of 32 and so more waves in flight)
constexpr int GEMV_ROWS = 32;
template <int QM>
__global__ __launch_bounds__(256) void gemv_rows_kernel(int64_t rows, int p, int q,
                                                        const double* __restrict__ A, int64_t lda,
                                                        const double* __restrict__ M,
                                                        double* __restrict__ out, int64_t ldo,
                                                        const double* __restrict__ E, int64_t lde,
                                                        const double* __restrict__ alpha_ptr,
                                                        int alpha_mode, Batch bat) {
  raise_wave_priority();
  __shared__ double Ms[128 * 4];
  const int prob = blockIdx.y;
  A += prob * bat.sA;
  M += prob * bat.sB;
  out += prob * bat.sC;
  if (E) E += prob * bat.sD;
  if (alpha_ptr) alpha_ptr += prob * bat.sE;
  for (int e = threadIdx.x; e < p * q; e += 256) Ms[e] = M[e];
  __syncthreads();
  const int lane = threadIdx.x % 64;
  double f = 1.0;
  if (alpha_mode == 1) f = 1.0 / *alpha_ptr;
  else if (alpha_mode == 2) f = 1.0 / sqrt(*alpha_ptr);
  // each wave takes 8 consecutive rows and issues their loads together
  const int64_t rbase = (int64_t)blockIdx.x * GEMV_ROWS + (threadIdx.x / 64) * 8;
  double acc[8][QM];
#pragma unroll
  for (int j = 0; j < 8; ++j)
#pragma unroll
    for (int c = 0; c < QM; ++c) acc[j][c] = 0.0;
  for (int l = lane; l < p; l += 64) {
    double mv[QM];
#pragma unroll
    for (int c = 0; c < QM; ++c) mv[c] = c < q ? Ms[l * q + c] : 0.0;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int64_t row = rbase + j;
      const double a = row < rows ? A[row * lda + l] : 0.0;
#pragma unroll
      for (int c = 0; c < QM; ++c) acc[j][c] += a * mv[c];
    }
  }
  // Sum each row's 64 lane partials by halving exchanges: at offset 32 a lane keeps the four
  // rows on its side of the offset and receives its partner's partials of them, then two rows
  // at 16 and one at 8, so that lane l holds row (l >> 3) & 7 summed over the lanes that share
  // l's bits 3-5; offsets 4, 2 and 1 finish the sum.  (Every index of acc is a compile-time
  // constant, so the array stays in registers.)
#pragma unroll
  for (int c = 0; c < QM; ++c) {
    if (c < q) {
      double v[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) v[j] = acc[j][c];
#pragma unroll
      for (int lev = 0; lev < 3; ++lev) {
        const int off = 32 >> lev, m = 4 >> lev;
        const bool upper = (lane & off) != 0;
#pragma unroll
        for (int i = 0; i < m; ++i) {
          const double give = upper ? v[i] : v[i + m];
          const double keep = upper ? v[i + m] : v[i];
          v[i] = keep + __shfl_xor(give, off);
        }
      }
#pragma unroll
      for (int off = 4; off > 0; off >>= 1) v[0] += __shfl_xor(v[0], off);
      acc[0][c] = v[0];
    }
  }
  const int64_t row = rbase + ((lane >> 3) & 7);
  if ((lane & 7) == 0 && row < rows) {
#pragma unroll
    for (int c = 0; c < QM; ++c) {
      if (c < q) {
        double v = acc[0][c];
        if (E) v += f * E[row * lde + c];
        out[row * ldo + c] = v;
      }
    }
  }
}

// ---------------------------------------------------------------- OUT = f(alpha) E + (A + delta A2) M
constexpr int M_T = 32;
__global__ __launch_bounds__(256) void gemm_rm_kernel(int64_t rows, int p, int q,
                                                      const double* __restrict__ A,
                                                      const double* __restrict__ A2,
                                                      const double* __restrict__ delta_ptr,
                                                      int64_t lda, const double* __restrict__ M,
                                                      double* __restrict__ out, int64_t ldo,
                                                      const double* __restrict__ E, int64_t lde,
                                                      const double* __restrict__ alpha_ptr,
                                                      int alpha_mode, Batch bat) {
  raise_wave_priority();
  __shared__ double As[M_T][M_T + 1];
  const int prob = blockIdx.z;
  A += prob * bat.sA;
  if (A2) A2 += prob * bat.sA;
  if (delta_ptr) delta_ptr += prob * bat.sE;
  M += prob * bat.sB;
  out += prob * bat.sC;
  if (E) E += prob * bat.sD;
  if (alpha_ptr) alpha_ptr += prob * bat.sE;
  __shared__ double Ms[M_T][M_T + 1];
  const int tc = threadIdx.x % M_T;
  const int tr = threadIdx.x / M_T;  // 0..7, rows tr*4 .. tr*4+3
  const int64_t row0 = (int64_t)blockIdx.y * M_T;
  const int col = blockIdx.x * M_T + tc;
  const double delta = (A2 && delta_ptr) ? *delta_ptr : 0.0;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int l0 = 0; l0 < p; l0 += M_T) {
    for (int e = threadIdx.x; e < M_T * M_T; e += 256) {
      const int a = e / M_T, b = e % M_T;
      const int64_t row = row0 + a;
      double v = 0.0;
      if (row < rows && l0 + b < p) {
        v = A[row * lda + l0 + b];
        if (A2) v += delta * A2[row * lda + l0 + b];
      }
      As[a][b] = v;
      Ms[a][b] = (l0 + a < p && blockIdx.x * M_T + b < q) ? M[(int64_t)(l0 + a) * q + blockIdx.x * M_T + b] : 0.0;
    }
    __syncthreads();
#pragma unroll 8
    for (int l = 0; l < M_T; ++l) {
      const double m = Ms[l][tc];
#pragma unroll
      for (int u = 0; u < 4; ++u) acc[u] += As[tr * 4 + u][l] * m;
    }
    __syncthreads();
  }
  if (col >= q) return;
  double f = 1.0;
  if (alpha_mode == 1) f = 1.0 / *alpha_ptr;
  else if (alpha_mode == 2) f = 1.0 / sqrt(*alpha_ptr);
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int64_t row = row0 + tr * 4 + u;
    if (row < rows) {
      double v = acc[u];
      if (E) v += f * E[row * lde + col];
      out[row * ldo + col] = v;
    }
  }
}

// ---------------------------------------------------------------- Nystrom core
// The r x r core lives in LDS as its upper triangle, packed row by row (element (i, j), i <= j,
// at i r - i (i + 1) / 2 + j): the Cholesky factor R overwrites it, then R^{-1} overwrites R in
// place, so the kernel needs about half the LDS of a full square (and finds room on a CU that
// a concurrent product kernel shares).
__device__ inline int up_idx(int i, int j, int r) { return i * r - (i * (i + 1)) / 2 + j; }

__global__ __launch_bounds__(1024) void nys_core_kernel(int r, const double* __restrict__ Mo,
                                                        const double* __restrict__ Qo, double eps,
                                                        double* __restrict__ Rinv,
                                                        double* __restrict__ Rg,
                                                        IterScalars* __restrict__ sc) {
  raise_wave_priority();
  __shared__ double C[RMAX * (RMAX + 1) / 2];
  {
    const int64_t off = (int64_t)blockIdx.x * r * r;
    Mo += off;
    Qo += off;
    Rinv += off;
    if (Rg) Rg += off;
    sc += blockIdx.x;
  }
  __shared__ double xt[RMAX];
  __shared__ double s_delta;
  const int tid = threadIdx.x;
  if (tid == 0) {
    double tr = 0.0;
    for (int i = 0; i < r; ++i) tr += Mo[i * r + i];
    s_delta = eps * tr;
  }
  __syncthreads();
  int ok = 0;
  int attempts = 0;
  for (; attempts <= 5; ++attempts) {
    const double delta = s_delta;
    for (int e = tid; e < r * r; e += 1024) {
      const int i = e / r, j = e % r;
      if (j >= i) C[up_idx(i, j, r)] = 0.5 * (Mo[i * r + j] + Mo[j * r + i]) + delta * Qo[i * r + j];
    }
    __syncthreads();
    // right-looking Cholesky C = R^T R (R upper), one barrier per column: column kk's
    // trailing update reads the unscaled row kk (C[i][j] -= C[kk][i] C[kk][j] / piv), and row
    // kk takes its final values, R[kk][kk] = sqrt(piv) and R[kk][j] = C[kk][j] / R[kk][kk], in
    // column kk + 1's phase, when no thread reads it any more.  The pivot test is uniform.
    const int ti = tid / 32, tj = tid % 32;
    double prev_dk = 0.0;
    bool bad = false;
    for (int kk = 0; kk < r; ++kk) {
      const double piv = C[up_idx(kk, kk, r)];
      if (!(piv > 0.0)) {
        bad = true;
        break;
      }
      if (kk > 0) {
        // row kk - 1: last changed by column kk - 2's update
        if (tid == 0) C[up_idx(kk - 1, kk - 1, r)] = prev_dk;
        for (int j = kk + tid; j < r; j += 1024) C[up_idx(kk - 1, j, r)] /= prev_dk;
      }
      const double inv_piv = 1.0 / piv;
      for (int i = kk + 1 + ti; i < r; i += 32) {
        const double ci = C[up_idx(kk, i, r)] * inv_piv;
        for (int j = kk + 1 + tj; j < r; j += 32)
          if (j >= i) C[up_idx(i, j, r)] -= ci * C[up_idx(kk, j, r)];
      }
      prev_dk = sqrt(piv);
      __syncthreads();
    }
    if (!bad) {
      if (tid == 0) C[up_idx(r - 1, r - 1, r)] = prev_dk;
      __syncthreads();
      ok = 1;
      break;
    }
    __syncthreads();
    if (tid == 0) s_delta *= 10.0;
    __syncthreads();
  }
  if (tid == 0) {
    sc->delta = s_delta;
    sc->not_pd = attempts > 0 ? 1 : 0;
    sc->failed = ok ? 0 : 1;
  }
  if (!ok) {
    for (int e = tid; e < r * r; e += 1024) {
      Rinv[e] = (e / r == e % r) ? 1.0 : 0.0;
      if (Rg) Rg[e] = Rinv[e];
    }
    return;
  }
  if (Rg)
    for (int e = tid; e < r * r; e += 1024) {
      const int i = e / r, j = e % r;
      Rg[e] = j >= i ? C[up_idx(i, j, r)] : 0.0;
    }
  // X = R^{-1} (upper) in place, rows i from the bottom: X[i][j] = -(sum_{l=i+1..j} R[i][l]
  // X[l][j]) / R[i][i] uses row i of R (still in place) and the rows below it (already X);
  // the new row goes through xt and is written back after a barrier.  8 threads per column.
  const int j = tid / 8, part = tid % 8;
  for (int i = r - 1; i >= 0; --i) {
    if (j < r && j > i) {
      double s = 0.0;
      for (int l = i + 1 + part; l <= j; l += 8) s += C[up_idx(i, l, r)] * C[up_idx(l, j, r)];
      s += __shfl_xor(s, 1, 8);
      s += __shfl_xor(s, 2, 8);
      s += __shfl_xor(s, 4, 8);
      if (part == 0) xt[j] = -s / C[up_idx(i, i, r)];
    }
    __syncthreads();
    if (j < r && j >= i && part == 0) {
      if (j == i) C[up_idx(i, i, r)] = 1.0 / C[up_idx(i, i, r)];
      else C[up_idx(i, j, r)] = xt[j];
    }
    __syncthreads();
  }
  for (int e = tid; e < r * r; e += 1024) {
    const int a = e / r, b = e % r;
    Rinv[e] = a <= b ? C[up_idx(a, b, r)] : 0.0;
  }
}

// ---------------------------------------------------------------- Jacobi eigensolver
// Parallel cyclic Jacobi: each step applies r/2 disjoint rotations (round-robin pairing),
// H <- J^T H J, as independent 2x2-block updates (block (a, b) mixes rows of pair a with
// columns of pair b), one LDS pass per step over the upper triangle only.
constexpr int JAC_MAX_SWEEPS = 16;

__device__ inline int rr_index(int i, int step, int rp) {
  // circle method: player 0 fixed, the others rotate by `step`
  return i == 0 ? 0 : 1 + (i - 1 + step) % (rp - 1);
}

// Symmetric storage: the upper triangle of the (padded) rp x rp matrix, row-major, so that
// element (i, j), i <= j, sits at i rp - i (i + 1) / 2 + j.  A step updates each unordered pair
// of rotation pairs {a, b} once (a <= b); its four entries are distinct stored elements.
__device__ inline int sym_idx(int i, int j, int rp) {
  if (i > j) {
    const int t = i;
    i = j;
    j = t;
  }
  return i * rp - (i * (i + 1)) / 2 + j;
}

// The 2x2-block update J_a^T H J_b of the block of rotation pairs (a, b): rows mixed by
// (ca, sa), then columns by (cb, sb).
__device__ inline void jac_block(double ca, double sa, double cb, double sb, double h11, double h12,
                                 double h21, double h22, double& n11, double& n12, double& n21,
                                 double& n22) {
  const double r11 = ca * h11 - sa * h21, r12 = ca * h12 - sa * h22;
  const double r21 = sa * h11 + ca * h21, r22 = sa * h12 + ca * h22;
  n11 = cb * r11 - sb * r12;
  n12 = sb * r11 + cb * r12;
  n21 = cb * r21 - sb * r22;
  n22 = sb * r21 + cb * r22;
}

// The rotation (c, s) that annihilates apq, or (1, 0) below the threshold (returns whether it
// rotates).  t = tan of the angle, the root of smaller magnitude of t^2 + 2 tau t - 1 = 0 with
// tau = (aqq - app) / (2 apq): sgn(tau) / (|tau| + sqrt(1 + tau^2))
// = 2 |apq| sgn(tau) / (|d| + sqrt(d^2 + 4 apq^2)) with d = aqq - app (one division fewer;
// sgn(0) = +1).  It is formed whether or not the rotation is taken, so that the threshold's
// square root runs beside it.
__device__ inline bool jac_rotation(double apq, double app, double aqq, double abs_floor, double& c,
                                    double& s) {
  const double d = aqq - app;
  const double tt = 2.0 * fabs(apq) / (fabs(d) + sqrt(d * d + 4.0 * apq * apq));
  const double t = (d == 0.0 || ((d > 0.0) == (apq > 0.0))) ? tt : -tt;
  const double ct = 1.0 / sqrt(1.0 + t * t);
  if (fabs(apq) > fmax(1e-15 * sqrt(fabs(app * aqq)), abs_floor)) {
    c = ct;
    s = t * ct;
    return true;
  }
  c = 1.0;
  s = 0.0;
  return false;
}

__global__ __launch_bounds__(1024) void jacobi_kernel(int r, const double* __restrict__ Hg,
                                                      double* __restrict__ evals,
                                                      double* __restrict__ rot,
                                                      IterScalars* __restrict__ sc,
                                                      int64_t rot_cap) {
  raise_wave_priority();
  __shared__ double H[RMAX * (RMAX + 1) / 2];
  Hg += (int64_t)blockIdx.x * r * r;
  evals += (int64_t)blockIdx.x * r;
  rot += (int64_t)blockIdx.x * rot_cap;
  sc += blockIdx.x;
  __shared__ double2 cs[RMAX / 2];  // (c, s) of each rotation pair of the step
  __shared__ int pq[RMAX / 2];      // its indices p | q << 16
  __shared__ int nrot;
  __shared__ double hmax;
  const int tid = threadIdx.x;
  const int rp = r + (r & 1);
  const int half = rp / 2;
  const int nblk = half * (half + 1) / 2;
  // the padded dummy index (odd r) has a zero row and column and is never rotated
  for (int i = tid; i < rp; i += 1024)
    for (int j = i; j < rp; ++j) H[sym_idx(i, j, rp)] = (i < r && j < r) ? Hg[i * r + j] : 0.0;
  // the pair-of-pairs blocks (a, b), a <= b, of this thread: blocks tid + 1024 u, the same
  // at every step (a thread without a block u takes (0, 0) and stores nothing for it)
  constexpr int JB = ((RMAX / 2) * (RMAX / 2 + 1) / 2 + 1023) / 1024;
  int blk_a[JB], blk_b[JB];
  bool blk_on[JB];
#pragma unroll
  for (int u = 0; u < JB; ++u) {
    const int e = tid + 1024 * u;
    int a = 0, rem = e < nblk ? e : 0;
    while (rem >= half - a) {
      rem -= half - a;
      ++a;
    }
    blk_a[u] = a;
    blk_b[u] = a + rem;
    blk_on[u] = e < nblk;
  }
  __syncthreads();
  if (tid == 0) {
    double m = 0.0;
    for (int i = 0; i < r; ++i) m = fmax(m, fabs(H[sym_idx(i, i, rp)]));
    hmax = m;
  }
  __syncthreads();
  const double abs_floor = 1e-300 + 1e-18 * hmax;
  int sweeps_used = 0;
  for (int sweep = 0; sweep < JAC_MAX_SWEEPS; ++sweep) {
    if (tid == 0) nrot = 0;
    __syncthreads();
    // the pair of rotation thread tid: indices rr_index(tid, step) and rr_index(rp - 1 - tid,
    // step), i.e. 1 + (offset + step) mod (rp - 1), kept as offsets that advance by one a step
    int oa = tid - 1, ob = rp - 2 - tid;
    for (int step = 0; step < rp - 1; ++step) {
      if (tid < half) {
        const int a = tid == 0 ? 0 : 1 + oa, b = 1 + ob;
        oa = oa + 1 == rp - 1 ? 0 : oa + 1;
        ob = ob + 1 == rp - 1 ? 0 : ob + 1;
        const int p = a < b ? a : b, q = a < b ? b : a;
        double c = 1.0, s = 0.0;
        if (q < r) {
          const double apq = H[sym_idx(p, q, rp)];
          const double app = H[sym_idx(p, p, rp)], aqq = H[sym_idx(q, q, rp)];
          if (jac_rotation(apq, app, aqq, abs_floor, c, s)) atomicAdd(&nrot, 1);
        }
        cs[tid] = make_double2(c, s);
        pq[tid] = p | (q << 16);
        const int64_t slot = ((int64_t)sweep * (rp - 1) + step) * half + tid;
        rot[2 * slot] = c;
        rot[2 * slot + 1] = s;
      }
      __syncthreads();
      // one block after the other: its (c, s) pairs and indices in one round of LDS reads, its
      // four entries in a second (the register budget must leave the kernel room beside the
      // Step-I product on a CU)
#pragma unroll
      for (int u = 0; u < JB; ++u) {
        if (!blk_on[u]) continue;
        const double2 csa = cs[blk_a[u]], csb = cs[blk_b[u]];
        const int pqa = pq[blk_a[u]], pqb = pq[blk_b[u]];
        const double ca = csa.x, sa = csa.y, cb = csb.x, sb = csb.y;
        if (sa == 0.0 && sb == 0.0) continue;
        const int pa = pqa & 0xffff, qa = pqa >> 16, pb = pqb & 0xffff, qb = pqb >> 16;
        const int i11 = sym_idx(pa, pb, rp), i12 = sym_idx(pa, qb, rp);
        const int i21 = sym_idx(qa, pb, rp), i22 = sym_idx(qa, qb, rp);
        double n11, n12, n21, n22;
        jac_block(ca, sa, cb, sb, H[i11], H[i12], H[i21], H[i22], n11, n12, n21, n22);
        if (blk_a[u] == blk_b[u]) {
          // diagonal block (pa < qa): i12 == i21; the rotation annihilates the off-diagonal entry
          H[i11] = n11;
          H[i12] = sa != 0.0 ? 0.0 : n12;
          H[i22] = n22;
        } else {
          H[i11] = n11;
          H[i12] = n12;
          H[i21] = n21;
          H[i22] = n22;
        }
      }
      __syncthreads();
    }
    const int done = nrot;
    __syncthreads();
    if (done == 0) break;
    sweeps_used = sweep + 1;
  }
  for (int i = tid; i < r; i += 1024) evals[i] = H[sym_idx(i, i, rp)];
  if (tid == 0) sc->sweeps = sweeps_used;
}

// Whole-wave lane shifts of a double (DPP wave_shl:1 / wave_shr:1, vector-ALU moves): lane i
// receives lane i + 1's value (from_next) or lane i - 1's (from_prev); the end lane keeps its
// own.
__device__ inline double from_next(double x) {
  const int lo = __double2loint(x), hi = __double2hiint(x);
  return __hiloint2double(__builtin_amdgcn_update_dpp(hi, hi, 0x130, 0xf, 0xf, false),
                          __builtin_amdgcn_update_dpp(lo, lo, 0x130, 0xf, 0xf, false));
}
__device__ inline double from_prev(double x) {
  const int lo = __double2loint(x), hi = __double2hiint(x);
  return __hiloint2double(__builtin_amdgcn_update_dpp(hi, hi, 0x138, 0xf, 0xf, false),
                          __builtin_amdgcn_update_dpp(lo, lo, 0x138, 0xf, 0xf, false));
}

// V = J_1 J_2 ... applied to the identity.  Rows of V are independent: a workgroup of NW
// waves takes NW * RPW rows, each wave RPW of them in registers.  Lane k holds, for each of its
// rows, the two entries that rotation pair k mixes at the current step: seat k and seat
// rp - 1 - k of the round-robin schedule (index rr_index(seat, step)).  After every step the
// schedule moves each index by one seat among seats 1 .. rp - 1 (seat 0 stays), i.e. the first
// entries shift down by one lane and the second entries up by one lane (DPP moves), with the
// two ends exchanged; after whole sweeps the indices are back at their step-0 seats.  The
// workgroup reads the rotations once, ACC_CH steps at a time, through two LDS buffers: the
// next chunk is loaded into registers while the current one is applied, one barrier a chunk.
constexpr int ACC_CH = 16;
template <int RPW, int NW>
__global__ __launch_bounds__(NW * 64) void jacobi_accum_kernel(int r, const double* __restrict__ rot,
                                                               const IterScalars* __restrict__ sc,
                                                               double* __restrict__ V,
                                                               int64_t rot_cap) {
  raise_wave_priority();
  constexpr int NT = NW * 64;
  constexpr int PER_T = (ACC_CH * (RMAX / 2) + NT - 1) / NT;  // staged elements per thread
  __shared__ double2 rb[2][ACC_CH * (RMAX / 2)];
  rot += (int64_t)blockIdx.y * rot_cap;
  sc += blockIdx.y;
  V += (int64_t)blockIdx.y * r * r;
  const int tid = threadIdx.x;
  const int k = tid % 64;  // rotation pair (lanes >= half hold zeros)
  const int rp = r + (r & 1);
  const int half = rp / 2;
  const int row0 = (blockIdx.x * NW + tid / 64) * RPW;
  const int ia0 = k, ib0 = rp - 1 - k;  // step-0 indices of the two seats of pair k
  const bool live = k < half;
  double A[RPW], Bv[RPW];
#pragma unroll
  for (int j = 0; j < RPW; ++j) {
    A[j] = (live && row0 + j == ia0) ? 1.0 : 0.0;
    Bv[j] = (live && row0 + j == ib0) ? 1.0 : 0.0;
  }
  const int steps = sc->sweeps * (rp - 1);
  const int per_chunk = ACC_CH * half;
  const double2* rot2 = reinterpret_cast<const double2*>(rot);
  double2 nx[PER_T];
  // element e = tid + NT u of the chunk that starts at step g0 (clamped to the last step)
  auto fetch = [&](int g0) __attribute__((always_inline)) {
#pragma unroll
    for (int u = 0; u < PER_T; ++u) {
      const int e = tid + NT * u;
      const int ec = e < per_chunk ? e : 0;
      int g = g0 + ec / half;
      g = g < steps ? g : steps - 1;
      nx[u] = rot2[(int64_t)g * half + ec % half];
    }
  };
  auto stage = [&](int buf) __attribute__((always_inline)) {
#pragma unroll
    for (int u = 0; u < PER_T; ++u) {
      const int e = tid + NT * u;
      if (e < per_chunk) rb[buf][e] = nx[u];
    }
  };
  // offsets of the two seats in the rotating part: index = 1 + (off + step) mod (rp - 1)
  int oa = k - 1, ob = rp - 2 - k;
  const int kk = live ? k : 0;
  if (steps > 0) {
    fetch(0);
    stage(0);
  }
  __syncthreads();
  int cb = 0;
  for (int g0 = 0; g0 < steps; g0 += ACC_CH) {
    const bool more = g0 + ACC_CH < steps;
    if (more) fetch(g0 + ACC_CH);
#pragma unroll
    for (int u = 0; u < ACC_CH; ++u) {
      if (g0 + u < steps) {
        const double2 cs2 = rb[cb][u * half + kk];
        // indices of the two seats at this step (seat 0 is index 0 throughout)
        const int a = k == 0 ? 0 : 1 + oa, b = 1 + ob;
        // the rotation (v_p, v_q) <- (c v_p - s v_q, s v_p + c v_q) with the first seat holding
        // p (a < b) or q: A <- c A + s' B, B <- c B - s' A with s' = -s or +s.  A step without a
        // rotation has c = 1, s = 0 and leaves both unchanged.
        const double c = cs2.x, sf = a > b ? cs2.y : -cs2.y;
#pragma unroll
        for (int j = 0; j < RPW; ++j) {
          const double na = c * A[j] + sf * Bv[j], nb = c * Bv[j] - sf * A[j];
          A[j] = na;
          Bv[j] = nb;
        }
#pragma unroll
        for (int j = 0; j < RPW; ++j) {
          const double tA = from_next(A[j]), tB = from_prev(Bv[j]);
          const double nA = k == 0 ? A[j] : (k < half - 1 ? tA : Bv[j]);
          const double nB = k == 0 ? (half > 1 ? tA : Bv[j]) : tB;
          A[j] = nA;
          Bv[j] = nB;
        }
        oa = oa + 1 == rp - 1 ? 0 : oa + 1;
        ob = ob + 1 == rp - 1 ? 0 : ob + 1;
      }
    }
    if (more) stage(cb ^ 1);
    __syncthreads();
    cb ^= 1;
  }
#pragma unroll
  for (int j = 0; j < RPW; ++j) {
    const int row = row0 + j;
    if (live && row < r) {
      if (ia0 < r) V[(int64_t)row * r + ia0] = A[j];
      if (ib0 < r) V[(int64_t)row * r + ib0] = Bv[j];
    }
  }
}

__global__ void nys_finalize_kernel(int r, const double* __restrict__ evals,
                                    const double* __restrict__ V, int rho_rule, double lam,
                                    double rho_fixed, double* __restrict__ S,
                                    double* __restrict__ T, double* __restrict__ cinv,
                                    double* __restrict__ cisq, IterScalars* __restrict__ sc) {
  raise_wave_priority();
  __shared__ int perm[RMAX];
  {
    const int pb = blockIdx.x;
    evals += (int64_t)pb * r;
    V += (int64_t)pb * r * r;
    S += (int64_t)pb * r;
    T += (int64_t)pb * r * r;
    cinv += (int64_t)pb * r;
    cisq += (int64_t)pb * r;
    sc += pb;
  }
  __shared__ double sig2[RMAX];
  __shared__ double s_rho;
  const int i = threadIdx.x;
  const double delta = sc->delta;
  if (i < r) {
    const double e = evals[i];
    int rank = 0;
    for (int j = 0; j < r; ++j) {
      const double f = evals[j];
      rank += (f > e) || (f == e && j < i);
    }
    perm[rank] = i;
  }
  __syncthreads();
  if (i < r) {
    const int src = perm[i];
    const double e = evals[src];
    sig2[i] = e;
    S[i] = fmax(0.0, e - delta);
  }
  __syncthreads();
  if (i == 0) {
    s_rho = rho_rule == 0 ? lam + S[r - 1] : rho_fixed;
    sc->rho = s_rho;
  }
  __syncthreads();
  const double rho = s_rho;
  if (i < r) {
    const double si = S[i];
    cinv[i] = 1.0 / (si + rho) - 1.0 / rho;
    cisq[i] = 1.0 / sqrt(si + rho) - 1.0 / sqrt(rho);
    const double e = sig2[i];
    const double inv = e > 0.0 ? 1.0 / sqrt(e) : 0.0;
    const int src = perm[i];
    for (int l = 0; l < r; ++l) T[l * r + i] = V[l * r + src] * inv;
  }
}

// ---------------------------------------------------------------- powering reductions
// Randomized powering: v . z and z . z (the Rayleigh quotient and the norm) in one workgroup
// per problem, in a fixed order (strided partials per thread, then the 64 lanes of each wave,
// then the waves), then v = z / |z|.  The vectors have one block's b entries, so one launch
// does what a partial-sum, a final-sum and a scaling launch would.  v and z may be the same
// vector: every entry is read before the barrier that precedes the writes.
constexpr int DN_THREADS = 1024;
__global__ __launch_bounds__(DN_THREADS) void dots_normalize_kernel(int64_t n, const double* z,
                                                                    double* v,
                                                                    IterScalars* __restrict__ sc,
                                                                    int last) {
  raise_wave_priority();
  __shared__ double wa[DN_THREADS / 64], wb[DN_THREADS / 64];
  __shared__ double inv_s;
  z += (int64_t)blockIdx.x * n;
  v += (int64_t)blockIdx.x * n;
  sc += blockIdx.x;
  const int tid = threadIdx.x;
  double a = 0.0, b = 0.0;
  for (int64_t i = tid; i < n; i += DN_THREADS) {
    const double zi = z[i];
    a += v[i] * zi;
    b += zi * zi;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    a += __shfl_xor(a, off);
    b += __shfl_xor(b, off);
  }
  if (tid % 64 == 0) {
    wa[tid / 64] = a;
    wb[tid / 64] = b;
  }
  __syncthreads();
  if (tid == 0) {
    double sa = 0.0, sb = 0.0;
    for (int w = 0; w < DN_THREADS / 64; ++w) {
      sa += wa[w];
      sb += wb[w];
    }
    sc->rq = sa;
    sc->vnorm2 = sb;
    inv_s = 1.0 / sqrt(sb);
    if (last) {
      sc->lam_hat = sa;
      sc->eta = 1.0 / sa;
    }
  }
  __syncthreads();
  const double inv = inv_s;
  for (int64_t i = tid; i < n; i += DN_THREADS) v[i] = z[i] * inv;
}

// One step of randomized powering on M = P^{-1/2} (K + lambda I) P^{-1/2} carried as
// w = P^{-1/2} v (v the unit iterate): with u = (K + lambda I) w and y = P^{-1} u,
// v . M v = w . u and |M v|^2 = u . y, and the next w is y / sqrt(u . y) -- the same iterates
// as applying P^{-1/2} before and after the product, with one Woodbury apply per step instead
// of two.  One workgroup per problem; the sums in a fixed order as above.  y may equal u.
__global__ __launch_bounds__(DN_THREADS) void power_step_kernel(int64_t n, double* w,
                                                                const double* u, const double* y,
                                                                IterScalars* __restrict__ sc,
                                                                int last) {
  raise_wave_priority();
  __shared__ double wa[DN_THREADS / 64], wb[DN_THREADS / 64];
  __shared__ double inv_s;
  w += (int64_t)blockIdx.x * n;
  u += (int64_t)blockIdx.x * n;
  y += (int64_t)blockIdx.x * n;
  sc += blockIdx.x;
  const int tid = threadIdx.x;
  double a = 0.0, b = 0.0;
  for (int64_t i = tid; i < n; i += DN_THREADS) {
    const double ui = u[i];
    a += w[i] * ui;
    b += ui * y[i];
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    a += __shfl_xor(a, off);
    b += __shfl_xor(b, off);
  }
  if (tid % 64 == 0) {
    wa[tid / 64] = a;
    wb[tid / 64] = b;
  }
  __syncthreads();
  if (tid == 0) {
    double sa = 0.0, sb = 0.0;
    for (int q = 0; q < DN_THREADS / 64; ++q) {
      sa += wa[q];
      sb += wb[q];
    }
    sc->rq = sa;
    sc->vnorm2 = sb;
    inv_s = 1.0 / sqrt(sb);
    if (last) {
      sc->lam_hat = sa;
      sc->eta = 1.0 / sa;
    }
  }
  __syncthreads();
  const double inv = inv_s;
  for (int64_t i = tid; i < n; i += DN_THREADS) w[i] = y[i] * inv;
}

__global__ void woodbury_coefs_kernel(int r, const double* __restrict__ S, double rho, int power,
                                      double* __restrict__ coefs, IterScalars* __restrict__ sc) {
  const int i = threadIdx.x;
  if (i < r)
    coefs[i] = power == 0 ? 1.0 / (S[i] + rho) - 1.0 / rho : 1.0 / sqrt(S[i] + rho) - 1.0 / sqrt(rho);
  if (i == 0) sc->rho = rho;
}

}  // namespace

adasap_status_t woodbury_coefs(int r, const double* S, double rho, int power, double* coefs,
                               IterScalars* sc, hipStream_t s) {
  hipLaunchKernelGGL(woodbury_coefs_kernel, dim3(1), dim3(RMAX), 0, s, r, S, rho, power, coefs, sc);
  ADASAP_LAUNCH_CHECK();
  return ADASAP_OK;
}

adasap_status_t gram(int64_t rows, int p, int q, const void* A, DT at, int64_t lda, const void* B,
                     DT bt, int64_t ldb, double* P, const double* rowscale, DevBuf& part,
                     hipStream_t s, const Batch& bat) {
  const int NP = bat.P;
  if (q <= 4 && p <= 128) {
    int64_t chunk = (rows + 255) / 256;
    chunk = chunk < 64 ? 64 : (chunk + 1) / 2 * 2;
    int sp = (int)((rows + chunk - 1) / chunk);
    if (sp < 1) sp = 1;
    ADASAP_TRY(part.ensure((size_t)NP * sp * p * q * sizeof(double)));
    if (rows > 0) {
      hipLaunchKernelGGL(gramv_partial_kernel, dim3(sp, NP), dim3(256), 0, s, rows, p, q, A, at, lda,
                         B, bt, ldb, part.as<double>(), bat, chunk);
      ADASAP_LAUNCH_CHECK();
    } else {
      ADASAP_HIP(hipMemsetAsync(part.p, 0, (size_t)NP * p * q * sizeof(double), s));
    }
    if (sp >= 32)
      hipLaunchKernelGGL(gram_reduce_tree_kernel, dim3(p * q, NP), dim3(256), 0, s,
                         part.as<double>(), sp, p, q, rowscale, P, bat);
    else
      hipLaunchKernelGGL(gram_reduce_kernel, dim3((p * q + 255) / 256, NP), dim3(256), 0, s,
                         part.as<double>(), sp, p, q, rowscale, P, bat);
    ADASAP_LAUNCH_CHECK();
    return ADASAP_OK;
  }
  // row splits: about 256 workgroups per launch (it runs beside the Step-I product), or 2048
  // for a batch (eight per CU, since a batch's Grams run alone), at least 64 rows each
  const int tiles = ((q + G_T - 1) / G_T) * ((p + G_T - 1) / G_T);
  const int64_t target = NP > 1 ? 2048 : 256;
  int64_t want = (target + (int64_t)tiles * NP - 1) / ((int64_t)tiles * NP);
  const int64_t most = (rows + 63) / 64;
  if (want > most) want = most;
  if (want < 1) want = 1;
  int64_t chunk = (rows + want - 1) / want;
  chunk = (chunk + G_ROWS - 1) / G_ROWS * G_ROWS;
  if (chunk < G_ROWS) chunk = G_ROWS;
  const int splits = (int)((rows + chunk - 1) / chunk > 0 ? (rows + chunk - 1) / chunk : 1);
  ADASAP_TRY(part.ensure((size_t)NP * splits * p * q * sizeof(double)));
  const dim3 grid((q + G_T - 1) / G_T, (p + G_T - 1) / G_T, splits * NP);
  hipLaunchKernelGGL(gram_partial_kernel, grid, dim3(256), 0, s, rows, p, q, A, at, lda, B, bt,
                     ldb, part.as<double>(), splits, chunk, bat);
  ADASAP_LAUNCH_CHECK();
  hipLaunchKernelGGL(gram_reduce_kernel, dim3((p * q + 255) / 256, NP), dim3(256), 0, s,
                     part.as<double>(), splits, p, q, rowscale, P, bat);
  ADASAP_LAUNCH_CHECK();
  return ADASAP_OK;
}

adasap_status_t gemm_rm(int64_t rows, int p, int q, const double* A, const double* A2,
                        const double* delta_ptr, int64_t lda, const double* M, double* out,
                        int64_t ldo, const double* E, int64_t lde, const double* alpha_ptr,
                        int alpha_mode, hipStream_t s, const Batch& bat) {
  if (rows <= 0) return ADASAP_OK;
  if (q <= 4 && p <= 128 && A2 == nullptr) {
    const dim3 grid((unsigned)((rows + GEMV_ROWS - 1) / GEMV_ROWS), bat.P);
    if (q == 1)
      hipLaunchKernelGGL(gemv_rows_kernel<1>, grid, dim3(256), 0, s, rows, p, q, A, lda, M, out, ldo,
                         E, lde, alpha_ptr, alpha_mode, bat);
    else
      hipLaunchKernelGGL(gemv_rows_kernel<4>, grid, dim3(256), 0, s, rows, p, q, A, lda, M, out, ldo,
                         E, lde, alpha_ptr, alpha_mode, bat);
    ADASAP_LAUNCH_CHECK();
    return ADASAP_OK;
  }
  const dim3 grid((q + M_T - 1) / M_T, (unsigned)((rows + M_T - 1) / M_T), bat.P);
  hipLaunchKernelGGL(gemm_rm_kernel, grid, dim3(256), 0, s, rows, p, q, A, A2, delta_ptr, lda, M,
                     out, ldo, E, lde, alpha_ptr, alpha_mode, bat);
  ADASAP_LAUNCH_CHECK();
  return ADASAP_OK;
}

adasap_status_t nys_core(int r, const double* Mo, const double* Qo, double eps, double* Rinv,
                         double* Rscratch, IterScalars* sc, hipStream_t s, int P) {
  if (r < 1 || r > RMAX) {
    set_error("nys_core: rank must be in [1, 128]");
    return ADASAP_ERR_INVALID_ARG;
  }
  hipLaunchKernelGGL(nys_core_kernel, dim3(P), dim3(1024), 0, s, r, Mo, Qo, eps, Rinv, Rscratch, sc);
  ADASAP_LAUNCH_CHECK();
  return ADASAP_OK;
}

size_t jacobi_rot_capacity(int r) {
  const int rp = r + (r & 1);
  return (size_t)JAC_MAX_SWEEPS * (rp - 1) * (rp / 2) * 2;
}

adasap_status_t jacobi_eig(int r, const double* H, double* evals, double* V, double* rot_buf,
                           IterScalars* sc, hipStream_t s, int P) {
  if (r < 1 || r > RMAX) {
    set_error("jacobi_eig: size must be in [1, 128]");
    return ADASAP_ERR_INVALID_ARG;
  }
  if (r == 1) {
    // 1 x 1: eigenvalue H, eigenvector 1
    std::vector<double> ones((size_t)P, 1.0);
    ADASAP_HIP(hipMemcpyAsync(evals, H, sizeof(double) * P, hipMemcpyDeviceToDevice, s));
    ADASAP_HIP(hipMemcpyAsync(V, ones.data(), sizeof(double) * P, hipMemcpyHostToDevice, s));
    ADASAP_HIP(hipStreamSynchronize(s));
    return ADASAP_OK;
  }
  const int64_t cap = (int64_t)jacobi_rot_capacity(r);
  hipLaunchKernelGGL(jacobi_kernel, dim3(P), dim3(1024), 0, s, r, H, evals, rot_buf, sc, cap);
  ADASAP_LAUNCH_CHECK();
  // one problem: workgroups of 4 waves x 2 rows spread the rows over many CUs (its chain runs
  // beside the Step-I product and is latency-bound); a batch: 16 waves x 4 rows, one workgroup
  // per 64 rows, so that each problem's rotations are read once or twice
  if (P == 1)
    hipLaunchKernelGGL((jacobi_accum_kernel<2, 4>), dim3((r + 7) / 8, P), dim3(256), 0, s, r,
                       rot_buf, sc, V, cap);
  else
    hipLaunchKernelGGL((jacobi_accum_kernel<4, 16>), dim3((r + 63) / 64, P), dim3(1024), 0, s, r,
                       rot_buf, sc, V, cap);
  ADASAP_LAUNCH_CHECK();
  return ADASAP_OK;
}

adasap_status_t nys_finalize(int r, const double* evals, const double* V, int rho_rule,
                             double lam, double rho_fixed, double* S, double* T, double* cinv,
                             double* cisq, IterScalars* sc, hipStream_t s, int P) {
  hipLaunchKernelGGL(nys_finalize_kernel, dim3(P), dim3(RMAX), 0, s, r, evals, V, rho_rule, lam,
                     rho_fixed, S, T, cinv, cisq, sc);
  ADASAP_LAUNCH_CHECK();
  return ADASAP_OK;
}

adasap_status_t normalize_inplace(int64_t b, double* v, IterScalars* sc, DevBuf& part,
                                  hipStream_t s, int P) {
  (void)part;
  return dots_normalize(b, v, v, sc, 0, s, P);
}

adasap_status_t power_step(int64_t b, double* w, const double* u, const double* y, IterScalars* sc,
                           int last, hipStream_t s, int P) {
  hipLaunchKernelGGL(power_step_kernel, dim3(P), dim3(DN_THREADS), 0, s, b, w, u, y, sc, last);
  ADASAP_LAUNCH_CHECK();
  return ADASAP_OK;
}

adasap_status_t dots_normalize(int64_t b, const double* z, double* v, IterScalars* sc, int last,
                               hipStream_t s, int P) {
  hipLaunchKernelGGL(dots_normalize_kernel, dim3(P), dim3(DN_THREADS), 0, s, b, z, v, sc, last);
  ADASAP_LAUNCH_CHECK();
  return ADASAP_OK;
}

}  // namespace adasap
