// Matrix-core kernel-block products for gfx950 (v_mfma_f32_16x16x32_f16).
//
// Squared distances.  Points are centred (mean mu) and scaled by sigma, x~ = sigma (x - mu),
// and split into float16 parts x~ = hi + lo.  With the norm term nx = |hi + lo|^2 / 2 split
// into three float16 parts (n1 + n2 + n3 = -nx), a column vector
//     [y_hi | y_lo | y_hi | ny1 ny2 ny3 | 1 1 1]
// dotted with a row vector
//     [x_hi | x_hi | x_lo | 1 1 1 | nx1 nx2 nx3]
// gives y_hi.x_hi + y_lo.x_hi + y_hi.x_lo - ny - nx = -sigma^2 |x - y|^2 / 2 up to the
// dropped lo.lo term (relative 2^-22), all on the matrix cores with float32 accumulation.
// With sigma^2 = log2(e)/ell^2 this is the RBF exponent for exp2; with sigma^2 = 2/ell^2 it is
// -(r/ell)^2 for the Matern family.  3d + 6 <= 32 needs one K-step of 32, d <= 16 two.
//
// Tiles.  A workgroup is 4 waves; each wave owns RT row tiles of 16 rows.  Columns stream
// through LDS in tiles of 32 (double buffered).  For each 16x16 (column x row) block the
// distance MFMA leaves lane l with columns 4(l/16)+0..3 of its column half and row l%16.
// The eight kernel values of a lane (two column halves) form the B operand of the next MFMA
// directly (K index = column slot), so the kernel block never leaves registers; the right-hand
// side tile is stored pre-permuted in the matching slot order.
//   MODE_F16   K and R in float16, one MFMA per (row tile, 16 right-hand sides); with 17 to
//              64 right-hand sides the same product runs on 32x32x16 MFMAs (MODE_F16W, below)
//   MODE_F16X3 K = K_hi + K_lo and R = R_hi + R_lo, three MFMAs (hi.hi + lo.hi + hi.lo)
//   MODE_F32V  K in float32 times float32 R on the vector ALUs (k <= 4); single and batched
//              products take the distances on 32x32x16 MFMAs (mkv_kernel, below), the
//              persistent batched Step I on the 16x16x32 form
// The column range is split over workgroups; partial sums are added in a fixed order.
#include <cmath>
#include <type_traits>

#include "mfma.h"
#include "kfun.h"

namespace adasap {

namespace {

typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef float f16v __attribute__((ext_vector_type(16)));

constexpr int TILE = 32;      // columns per tile
constexpr int WAVES = 4;      // waves per workgroup
constexpr int MODE_F16 = 0, MODE_F16X3 = 1, MODE_F32V = 2;
// MODE_F16 on 32x32x16 MFMAs ("wide" tiles), for 17 to 64 right-hand sides
constexpr int MODE_F16W = 3;
constexpr int ROWVEC = 64;    // float16 entries stored per point (two K-steps)

__device__ inline f4 mfma16(half8 a, half8 b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
}

__device__ inline f16v mfma32(half8 a, half8 b, f16v c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
}

// Wide tiles: column (within the tile) of index kappa of K-slice t.  The 32x32x16 MFMA leaves
// lane l of a 32 x 32 (column x row) distance block with row l % 32 and, in register r, column
// 8 (r / 4) + 4 (l / 32) + r % 4; registers 8t..8t+7 are the B operand of K-slice t of the
// K Z product (index kappa = 8 (l / 32) + j), so the right-hand side is packed in this order.
__host__ __device__ constexpr int wide_col(int t, int kappa) {
  return 16 * t + 8 * ((kappa % 8) / 4) + 4 * (kappa / 8) + kappa % 4;
}

// ---------------------------------------------------------------- packing
__global__ __launch_bounds__(256) void mean_partial_kernel(const void* __restrict__ X, DT xt,
                                                           int64_t n, int d,
                                                           double* __restrict__ part) {
  // block b sums rows [b*4096, ...): thread t takes coordinate t % d of rows t / d, t / d + 256 / d,
  // ...; the row groups are then added in a fixed order
  __shared__ double red[256];
  const int64_t r0 = (int64_t)blockIdx.x * 4096;
  const int64_t r1 = r0 + 4096 < n ? r0 + 4096 : n;
  const int tid = threadIdx.x;
  const int rstep = 256 / d, f = tid % d, rg = tid / d;
  double s = 0.0;
  if (rg < rstep)
    for (int64_t r = r0 + rg; r < r1; r += rstep)
      s += xt == DT::F64 ? static_cast<const double*>(X)[r * d + f]
                         : (double)static_cast<const float*>(X)[r * d + f];
  red[tid] = s;
  __syncthreads();
  if (tid < d) {
    double t = 0.0;
    for (int g = 0; g < rstep; ++g) t += red[g * d + tid];
    part[(int64_t)blockIdx.x * d + tid] = t;
  }
}

__global__ void mean_final_kernel(const double* __restrict__ part, int nblk, int d, int64_t n,
                                  double* __restrict__ mu) {
  for (int f = threadIdx.x; f < d; f += blockDim.x) {
    double s = 0.0;
    for (int b = 0; b < nblk; ++b) s += part[(int64_t)b * d + f];
    mu[f] = s / (double)n;
  }
}

// row-format vectors of points (one thread per point); flag set if float16 would overflow
__global__ void rowpack_kernel(const void* __restrict__ X, DT xt, int64_t n, int64_t npad, int d,
                               const double* __restrict__ mu, double sigma,
                               _Float16* __restrict__ rowv, int* __restrict__ flag) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= npad) return;
  _Float16* o = rowv + i * ROWVEC;
  for (int e = 0; e < ROWVEC; ++e) o[e] = (_Float16)0.0f;
  if (i >= n) return;
  double nrm = 0.0;
  bool bad = false;
  for (int f = 0; f < d; ++f) {
    const double x = xt == DT::F64 ? static_cast<const double*>(X)[i * d + f]
                                   : (double)static_cast<const float*>(X)[i * d + f];
    const double xs = sigma * (x - mu[f]);
    bad |= !(fabs(xs) < 30000.0);
    const _Float16 hi = (_Float16)(float)xs;
    const _Float16 lo = (_Float16)(float)(xs - (double)(float)hi);
    const double xh = (double)(float)hi + (double)(float)lo;
    nrm += xh * xh;
    o[f] = hi;
    o[d + f] = hi;
    o[2 * d + f] = lo;
  }
  const double nx = -0.5 * nrm;
  bad |= !(fabs(nx) < 30000.0);
  const _Float16 n1 = (_Float16)(float)nx;
  const double r1 = nx - (double)(float)n1;
  const _Float16 n2 = (_Float16)(float)r1;
  const _Float16 n3 = (_Float16)(float)(r1 - (double)(float)n2);
  o[3 * d + 0] = (_Float16)1.0f;
  o[3 * d + 1] = (_Float16)1.0f;
  o[3 * d + 2] = (_Float16)1.0f;
  o[3 * d + 3] = n1;
  o[3 * d + 4] = n2;
  o[3 * d + 5] = n3;
  if (bad) atomicOr(flag, 1);
}

// column A-fragments of the points idx[0..cnt) (identity if idx == null), from row vectors.
// Column vector = [hi | lo | hi | n1 n2 n3 | 1 1 1]; fragment of tile T, half cs, K-step ks,
// lane l holds column T*32 + cs*16 + l%16, entries ks*32 + 8(l/16) + 0..7.
__global__ void colpack_kernel(const _Float16* __restrict__ rowv, const int64_t* __restrict__ idx,
                               int64_t cnt, int64_t ntiles, int d, int KS,
                               half8* __restrict__ colA, const int* __restrict__ dvec) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;  // one fragment per thread
  const int64_t total = ntiles * 2 * KS * 64;
  if (e >= total) return;
  // batch: problem blockIdx.y has its own index list, fragments and dimension
  if (idx) idx += (int64_t)blockIdx.y * cnt;
  colA += (int64_t)blockIdx.y * total;
  if (dvec) d = dvec[blockIdx.y];
  const int lane = (int)(e % 64);
  const int ks = (int)((e / 64) % KS);
  const int cs = (int)((e / (64 * KS)) % 2);
  const int64_t T = e / (64 * KS * 2);
  const int64_t c = T * TILE + cs * 16 + lane % 16;
  half8 v;
  if (c >= cnt) {
    for (int j = 0; j < 8; ++j) v[j] = (_Float16)0.0f;
  } else {
    const _Float16* rv = rowv + (idx ? idx[c] : c) * ROWVEC;
    for (int j = 0; j < 8; ++j) {
      const int kk = ks * 32 + 8 * (lane / 16) + j;
      _Float16 val = (_Float16)0.0f;
      if (kk < d) val = rv[kk];                          // hi
      else if (kk < 2 * d) val = rv[2 * d + (kk - d)];   // lo
      else if (kk < 3 * d) val = rv[kk - 2 * d];         // hi
      else if (kk < 3 * d + 3) val = rv[3 * d + 3 + (kk - 3 * d)];  // n1 n2 n3
      else if (kk < 3 * d + 6) val = (_Float16)1.0f;
      v[j] = val;
    }
  }
  colA[e] = v;
}

// per-column maxima of |R| (rows x k, type rt), partials per 4096 rows; the block's threads
// sweep the chunk in memory order and combine through integer maxima of the float bits
// (non-negative floats order like their bit patterns)
__global__ __launch_bounds__(256) void colmax_partial_kernel(const void* __restrict__ R, DT rt,
                                                             int64_t rows, int k, int64_t ldr,
                                                             float* __restrict__ part, int64_t rpb) {
  __shared__ unsigned int mx[128];
  R = static_cast<const char*>(R) + (int64_t)blockIdx.y * rows * ldr * (rt == DT::F64 ? 8 : 4);
  part += (int64_t)blockIdx.y * gridDim.x * k;
  for (int c = threadIdx.x; c < k; c += 256) mx[c] = 0u;
  __syncthreads();
  const int64_t r0 = (int64_t)blockIdx.x * rpb;
  const int64_t r1 = r0 + rpb < rows ? r0 + rpb : rows;
  const int64_t cnt = (r1 - r0) * k;
  if (256 % k == 0) {
    // thread t reads column t % k of rows t / k, t / k + 256 / k, ...: a register maximum
    const int c = threadIdx.x % k;
    const int rstep = 256 / k;
    float m = 0.0f;
    if (rt == DT::F64) {
      const double* Rd = static_cast<const double*>(R);
      for (int64_t row = r0 + threadIdx.x / k; row < r1; row += rstep) {
        const float a = (float)fabs(Rd[row * ldr + c]);
        m = fmaxf(m, isfinite(a) ? a : 3.0e38f);
      }
    } else {
      const float* Rf = static_cast<const float*>(R);
      for (int64_t row = r0 + threadIdx.x / k; row < r1; row += rstep) {
        const float a = fabsf(Rf[row * ldr + c]);
        m = fmaxf(m, isfinite(a) ? a : 3.0e38f);
      }
    }
    atomicMax(&mx[c], __float_as_uint(m));
  } else {
    for (int64_t e = threadIdx.x; e < cnt; e += 256) {
      const int64_t row = r0 + e / k;
      const int c = (int)(e % k);
      const double v = rt == DT::F64 ? static_cast<const double*>(R)[row * ldr + c]
                                     : (double)static_cast<const float*>(R)[row * ldr + c];
      const float a = (float)fabs(v);
      atomicMax(&mx[c], __float_as_uint(isfinite(a) ? a : 3.0e38f));
    }
  }
  __syncthreads();
  for (int c = threadIdx.x; c < k; c += 256) part[(int64_t)blockIdx.x * k + c] = __uint_as_float(mx[c]);
}

// scale[c] = power of two with max|R[:, c]| / scale <= 2^14 (scale >= 2^-60), 1 if the column is 0.
// One block per (column, problem): a strided maximum over the partials, then a tree.
__global__ __launch_bounds__(256) void colmax_final_kernel(const float* __restrict__ part, int nblk,
                                                           int k, float* __restrict__ scale) {
  __shared__ float red[256];
  const int c = blockIdx.x;
  part += (int64_t)blockIdx.y * nblk * k;
  scale += (int64_t)blockIdx.y * k;
  float m = 0.0f;
  for (int b = threadIdx.x; b < nblk; b += 256) m = fmaxf(m, part[(int64_t)b * k + c]);
  red[threadIdx.x] = m;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + h]);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    m = red[0];
    float sc = 1.0f;
    if (m > 0.0f && isfinite(m)) {
      int ex;
      frexpf(m, &ex);  // m = f 2^ex, f in [0.5, 1)
      int p = ex - 14;
      if (p < -60) p = -60;
      sc = ldexpf(1.0f, p);
    }
    scale[c] = sc;
  }
}

// rows per block of the column-maximum partials: at least 64, about 2048 blocks
inline int64_t colmax_rows_per_block(int64_t rows) {
  int64_t rpb = (rows + 2047) / 2048;
  rpb = (rpb + 63) / 64 * 64;
  return rpb < 64 ? 64 : rpb;
}

// float16 right-hand-side fragments: tile T, tile q of 16 columns, part (hi, lo), lane, slot m
// slot m of lane l is column 4(l/16)+m (m < 4) or 16+4(l/16)+m-4 of the tile
__device__ inline int slot_col(int lane, int m) {
  return m < 4 ? 4 * (lane / 16) + m : 16 + 4 * (lane / 16) + (m - 4);
}

__global__ void rhspack16_kernel(const void* __restrict__ R, DT rt, int64_t rows, int k,
                                 int64_t ldr, const int64_t* __restrict__ idx,
                                 const float* __restrict__ scale, int64_t ntiles, int NQ, int parts,
                                 half8* __restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t total = ntiles * NQ * 64;
  if (e >= total) return;
  const int lane = (int)(e % 64);
  const int q = (int)((e / 64) % NQ);
  const int64_t T = e / (64 * NQ);
  const int rhs = q * 16 + lane % 16;
  R = static_cast<const char*>(R) + (int64_t)blockIdx.y * rows * ldr * (rt == DT::F64 ? 8 : 4);
  scale += (int64_t)blockIdx.y * k;
  out += (int64_t)blockIdx.y * ntiles * NQ * parts * 64;
  half8 hi, lo;
  const float inv = rhs < k ? 1.0f / scale[rhs] : 0.0f;
  // branch-free gathers (invalid slots read element 0 and are zeroed), so that the eight
  // loads of a thread are in flight together
  int64_t off[8];
  bool ok[8];
#pragma unroll
  for (int m = 0; m < 8; ++m) {
    const int64_t col = T * TILE + slot_col(lane, m);
    ok[m] = col < rows && rhs < k;
    const int64_t src = idx ? idx[ok[m] ? col : 0] : col;
    off[m] = ok[m] ? src * ldr + rhs : 0;
  }
  double x[8];
  if (rt == DT::F64) {
    const double* Rd = static_cast<const double*>(R);
#pragma unroll
    for (int m = 0; m < 8; ++m) x[m] = Rd[off[m]];
  } else {
    const float* Rf = static_cast<const float*>(R);
#pragma unroll
    for (int m = 0; m < 8; ++m) x[m] = (double)Rf[off[m]];
  }
#pragma unroll
  for (int m = 0; m < 8; ++m) {
    const float v = ok[m] ? (float)(x[m] * (double)inv) : 0.0f;
    const _Float16 h = (_Float16)v;
    hi[m] = h;
    lo[m] = (_Float16)(v - (float)h);
  }
  const int64_t base = (T * NQ + q) * parts;
  out[(base + 0) * 64 + lane] = hi;
  if (parts == 2) out[(base + 1) * 64 + lane] = lo;
}

// float16 right-hand side for wide tiles: per tile, NQW blocks of 32 right-hand sides and two
// K-slices of 16 columns, lane l holding right-hand side 32q + l % 32 and the eight columns
// wide_col(t, 8 (l / 32) + j), scaled as rhspack16_kernel does
__global__ void rhspackw_kernel(const void* __restrict__ R, DT rt, int64_t rows, int k,
                                int64_t ldr, const float* __restrict__ scale, int64_t ntiles,
                                int NQW, half8* __restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= ntiles * NQW * 128) return;
  const int lane = (int)(e % 64);
  const int t = (int)((e / 64) % 2);
  const int q = (int)((e / 128) % NQW);
  const int64_t T = e / (128 * (int64_t)NQW);
  const int rhs = q * 32 + lane % 32;
  const float inv = rhs < k ? 1.0f / scale[rhs] : 0.0f;
  int64_t off[8];
  bool ok[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const int64_t col = T * TILE + wide_col(t, 8 * (lane / 32) + j);
    ok[j] = col < rows && rhs < k;
    off[j] = ok[j] ? col * ldr + rhs : 0;
  }
  double x[8];
  if (rt == DT::F64) {
    const double* Rd = static_cast<const double*>(R);
#pragma unroll
    for (int j = 0; j < 8; ++j) x[j] = Rd[off[j]];
  } else {
    const float* Rf = static_cast<const float*>(R);
#pragma unroll
    for (int j = 0; j < 8; ++j) x[j] = (double)Rf[off[j]];
  }
  half8 h;
#pragma unroll
  for (int j = 0; j < 8; ++j) h[j] = (_Float16)(ok[j] ? (float)(x[j] * (double)inv) : 0.0f);
  out[((T * NQW + q) * 2 + t) * 64 + lane] = h;
}

// float32 right-hand side, padded to ntiles*32 rows and KC columns
template <int KC>
__global__ void rhspack32_kernel(const void* __restrict__ R, DT rt, int64_t rows, int k,
                                 int64_t ldr, const int64_t* __restrict__ idx, int64_t npad,
                                 float* __restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= npad * KC) return;
  R = static_cast<const char*>(R) + (int64_t)blockIdx.y * rows * ldr * (rt == DT::F64 ? 8 : 4);
  out += (int64_t)blockIdx.y * npad * KC;
  const int64_t i = e / KC;
  const int c = (int)(e % KC);
  float v = 0.0f;
  if (i < rows && c < k) {
    const int64_t src = idx ? idx[i] : i;
    v = rt == DT::F64 ? (float)static_cast<const double*>(R)[src * ldr + c]
                      : static_cast<const float*>(R)[src * ldr + c];
  }
  out[e] = v;
}

// ---------------------------------------------------------------- the product kernel
template <int KERN>
__device__ inline float kval(float s, float p) {
  // s = sigma-scaled exponent: RBF: exp2 argument; Matern: -(r/ell)^2
  if constexpr (KERN == ADASAP_RBF) {
    return __builtin_amdgcn_exp2f(s);
  } else {
    // a = p r / ell from s = -(r/ell)^2: the hardware square root (one instruction, within
    // 1 ulp) of |s| (a free source modifier).  The correctly rounded sqrtf and a clamp at
    // zero expand to about a dozen vector instructions, which made the Matern products
    // issue-bound on the vector ALUs.  s > 0 only where rounding of the split distance left
    // r^2 slightly negative; |s| is then within that rounding error of r^2.
    const float a = __builtin_amdgcn_sqrtf(__builtin_fabsf(s)) * p;  // p = 1, sqrt(3) or sqrt(5)
    const float e = __builtin_amdgcn_exp2f(-a * 1.4426950408889634f);
    if constexpr (KERN == ADASAP_MATERN12) return e;
    else if constexpr (KERN == ADASAP_MATERN32) return (1.0f + a) * e;
    else return (1.0f + a + a * a * (1.0f / 3.0f)) * e;
  }
}

struct MkItem {
  int prob, rw;     // problem and row workgroup
  int64_t T0, T1;   // column tiles [T0, T1) of that problem
  int slot, pad;    // partial-sum slot: start[prob] + rw * chunks[prob] + T0 / chunk
};

// the work queue is cut into one contiguous range per XCD; the range counters sit 128 bytes
// apart
constexpr int QXCDS = 8;
constexpr int QCOUNTER_STRIDE = 32;
static_assert(sizeof(MfmaQueue::qbeg) / sizeof(int) == QXCDS + 1, "one item range per XCD");

struct MkArgs {
  const half8* colA;     // column fragments [ntiles][2][KS][64]
  const half8* rowv;     // row vectors [points][8] (64 float16 each)
  const int64_t* ridx;   // row point indices (null: rows 0..m-1)
  int64_t m;             // rows
  const void* rhs;       // packed right-hand side
  int64_t ntiles;        // column tiles in total
  int64_t tiles_per_split;
  int splits;
  int rwg;               // row workgroups
  int xcd_map;           // 1: split-major items grouped by XCD (grid a multiple of 8)
  float* part;           // [splits][m][k]
  int k;
  float p;               // Matern factor
  // batches of equal-shape problems (blockIdx.y = problem): per-problem strides
  int64_t bs_colA;       // half8
  int64_t bs_ridx;       // indices
  int64_t bs_rhs;        // bytes
  int64_t bs_part;       // floats
  // work-queue launches over problems of uneven size
  const MkItem* items;
  int nitems;
  int* counter;
  const int64_t* colA_off;  // per problem, half8
  const int64_t* rhs_off;   // per problem, bytes
  int qbeg[QXCDS + 1];      // items [qbeg[x], qbeg[x + 1]) are drained by the workgroups of XCD x
};

// row tiles per wave: four (each column fragment read from LDS feeds four row tiles), two
// for the products with more than 64 right-hand sides.  Measured at the 2M-point, 64-column
// shape: two row tiles at four waves per SIMD run 15% slower than four at two.
constexpr int rt_of(int mode, int nq) { return (mode != MODE_F32V && nq > 4) ? 2 : 4; }
// workgroups per CU the launch bounds ask for: two; four for the float32 vector mode (k <= 4,
// at most 128 VGPRs, more waves to hide the transcendental latency); one for the hi/lo
// products with eight column tiles of the Matern-3/2 and -5/2 kernels, whose registers do
// not fit two waves per SIMD without scratch
template <int KERN, int MODE, int NQ>
constexpr int mk_occupancy() {
  return MODE == MODE_F32V ? 4 : ((MODE == MODE_F16X3 && NQ > 7 && KERN >= 2) ? 1 : 2);
}

// f(integral_constant<int, 0>), ..., f(integral_constant<int, N - 1>): indices stay
// compile-time constants (a #pragma unroll loop over a register array can be left rolled,
// which moves the array to scratch memory)
template <int N, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (N > 0) {
    static_for<N - 1>(f);
    f(std::integral_constant<int, N - 1>{});
  }
}

template <int KS, int MODE, int NQ>
struct MkShape {
  static constexpr int A_FR = 2 * KS * 64;                                            // half8 per tile
  static constexpr int R_FR = MODE == MODE_F16 ? NQ * 64 : (MODE == MODE_F16X3 ? 2 * NQ * 64 : 0);
  static constexpr int R_F32 = MODE == MODE_F32V ? TILE * NQ : 0;                     // floats (NQ = KC)
  static constexpr int TOTAL16 = A_FR + R_FR + (R_F32 * 4) / 16;  // 16-byte words of one tile
  static constexpr int BUF_BYTES = ((TOTAL16 + 255) / 256) * 256 * 16;  // whole load rounds
};

// Streams column tiles [T0, T1) of one problem against the rows of row workgroup rw and
// writes the partial sums of rows row_base.. to out[(row - out_row0) * k + c].
template <int KS, int KERN, int MODE, int NQ, int RT>
__device__ void mk_tiles(const MkArgs& a, char* lds, const half8* colA_p, const void* rhs_p,
                         const int64_t* ridx, int rw, int64_t T0, int64_t T1, float* out,
                         int64_t out_row0) {
  using SH = MkShape<KS, MODE, NQ>;
  constexpr int A_FR = SH::A_FR, R_FR = SH::R_FR, R_F32 = SH::R_F32, TOTAL16 = SH::TOTAL16;
  constexpr int BUF_BYTES = SH::BUF_BYTES;
  const int tid = threadIdx.x;
  const int lane = tid % 64;
  const int wave = tid / 64;
  const int64_t row_base = ((int64_t)rw * WAVES + wave) * RT * 16;
  // row operands (constant over the column stream)
  half8 Bfr[RT][KS];
#pragma unroll
  for (int rt = 0; rt < RT; ++rt) {
    const int64_t row = row_base + rt * 16 + lane % 16;
    const int64_t pt = row < a.m ? (ridx ? ridx[row] : row) : (ridx ? ridx[0] : 0);
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) Bfr[rt][ks] = a.rowv[pt * 8 + ks * 4 + lane / 16];
  }
  // consume the row fragments once here, so the loads are complete before the column stream
  // starts and no wait for them lands inside the loop (where it would also wait for prefetches)
#pragma unroll
  for (int rt = 0; rt < RT; ++rt)
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) asm volatile("" ::"v"(Bfr[rt][ks]));

  f4 acc[RT][MODE == MODE_F32V ? 1 : NQ];
  float accv[RT][MODE == MODE_F32V ? NQ : 1];
#pragma unroll
  for (int rt = 0; rt < RT; ++rt) {
#pragma unroll
    for (int q = 0; q < (MODE == MODE_F32V ? 1 : NQ); ++q) acc[rt][q] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int c = 0; c < (MODE == MODE_F32V ? NQ : 1); ++c) accv[rt][c] = 0.f;
  }

  // cooperative tile loads (global -> registers -> LDS), two tiles ahead of the compute, one
  // barrier per tile: while the waves compute tile T from one LDS buffer, tile T+1 is written
  // to the other and tile T+2 is in flight in registers
  constexpr int LOADS16 = (A_FR + R_FR + (R_F32 * 4) / 16 + 255) / 256;
  // separate members rather than an array: an array of five 16-byte words is kept in scratch
  static_assert(LOADS16 <= 5, "tile loads per thread");
  struct Stage {
    uint4 w0, w1, w2, w3, w4;
  };
  auto word = [](Stage& st, auto uc) __attribute__((always_inline)) -> uint4& {
    constexpr int u = decltype(uc)::value;
    if constexpr (u == 0) return st.w0;
    else if constexpr (u == 1) return st.w1;
    else if constexpr (u == 2) return st.w2;
    else if constexpr (u == 3) return st.w3;
    else return st.w4;
  };
  // branch-free loads (one basic block, so the wait before each LDS store covers exactly the
  // older of the two register stages); lanes past the tile's data read a valid dummy address.
  // Stages are passed by value so that they stay in registers.
  auto gload = [&](int64_t T) __attribute__((always_inline)) -> Stage {
    Stage st;
    const uint4* ca = reinterpret_cast<const uint4*>(colA_p) + T * A_FR;
    const uint4* rb = reinterpret_cast<const uint4*>(rhs_p) + T * (R_FR + (R_F32 * 4) / 16);
    static_for<LOADS16>([&](auto uc) {
      constexpr int u = decltype(uc)::value;
      const int e = tid + u * 256;
      const uint4* src = e < A_FR ? ca + e : (e < TOTAL16 ? rb + (e - A_FR) : ca);
      word(st, uc) = *src;
    });
    return st;
  };
  auto sstore = [&](Stage st, int buf) __attribute__((always_inline)) {
    uint4* dst = reinterpret_cast<uint4*>(lds + buf * BUF_BYTES);
    static_for<LOADS16>([&](auto uc) {
      constexpr int u = decltype(uc)::value;
      dst[tid + u * 256] = word(st, uc);
    });
  };
  // float16 mode, software-pipelined over tiles: the K Z products of a tile run in the
  // compute step of the next one, from the K and right-hand-side fragments kept in registers,
  // so that they overlap the next tile's distances and exponentials instead of waiting for
  // this tile's.  Each accumulator still adds the tiles in order.  Zero fragments before the
  // first tile make the first (and, with no tiles, the only) deferred step add nothing.
  constexpr bool PIPE = MODE == MODE_F16;
  half8 Kp[PIPE ? RT : 1];
  half8 Rp[PIPE ? NQ : 1];
  static_for<PIPE ? RT : 1>([&](auto ic) {
    constexpr int i = decltype(ic)::value;
#pragma unroll
    for (int j = 0; j < 8; ++j) Kp[i][j] = (_Float16)0.0f;
  });
  static_for<PIPE ? NQ : 1>([&](auto ic) {
    constexpr int i = decltype(ic)::value;
#pragma unroll
    for (int j = 0; j < 8; ++j) Rp[i][j] = (_Float16)0.0f;
  });
  auto kz_deferred = [&]() __attribute__((always_inline)) {
    if constexpr (PIPE) {
      static_for<RT>([&](auto rc) {
        constexpr int rt = decltype(rc)::value;
        static_for<NQ>([&](auto qc) {
          constexpr int q = decltype(qc)::value;
          acc[rt][q] = mfma16(Rp[q], Kp[rt], acc[rt][q]);
        });
      });
    }
  };

  auto compute = [&](int buf) __attribute__((always_inline)) {
    const half8* Af = reinterpret_cast<const half8*>(lds + buf * BUF_BYTES);
    if constexpr (PIPE) {
      kz_deferred();
      const half8* Rf = reinterpret_cast<const half8*>(lds + buf * BUF_BYTES + A_FR * 16);
      static_for<NQ>([&](auto qc) {
        constexpr int q = decltype(qc)::value;
        Rp[q] = Rf[q * 64 + lane];
      });
    }
    half8 A[2][KS];
#pragma unroll
    for (int cs = 0; cs < 2; ++cs)
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) A[cs][ks] = Af[(cs * KS + ks) * 64 + lane];

#pragma unroll
    for (int rt = 0; rt < RT; ++rt) {
      f4 S0 = f4{0.f, 0.f, 0.f, 0.f}, S1 = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) {
        S0 = mfma16(A[0][ks], Bfr[rt][ks], S0);
        S1 = mfma16(A[1][ks], Bfr[rt][ks], S1);
      }
      float kv[8];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        kv[j] = kval<KERN>(S0[j], a.p);
        kv[4 + j] = kval<KERN>(S1[j], a.p);
      }
      if constexpr (MODE == MODE_F32V) {
        const float* zr = reinterpret_cast<const float*>(lds + buf * BUF_BYTES + A_FR * 16);
        const int g = lane / 16;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          const int col = j < 4 ? 4 * g + j : 16 + 4 * g + (j - 4);
#pragma unroll
          for (int c = 0; c < NQ; ++c) accv[rt][c] += kv[j] * zr[col * NQ + c];
        }
      } else {
        half8 Kh;
#pragma unroll
        for (int j = 0; j < 8; ++j) Kh[j] = (_Float16)kv[j];
        const half8* Rf = reinterpret_cast<const half8*>(lds + buf * BUF_BYTES + A_FR * 16);
        if constexpr (MODE == MODE_F16) {
          (void)Rf;
          Kp[rt] = Kh;
        } else {
          half8 Kl;
#pragma unroll
          for (int j = 0; j < 8; ++j) Kl[j] = (_Float16)(kv[j] - (float)Kh[j]);
#pragma unroll
          for (int q = 0; q < NQ; ++q) {
            const half8 Rh = Rf[(q * 2 + 0) * 64 + lane];
            const half8 Rl = Rf[(q * 2 + 1) * 64 + lane];
            acc[rt][q] = mfma16(Rh, Kh, acc[rt][q]);
            acc[rt][q] = mfma16(Rl, Kh, acc[rt][q]);
            acc[rt][q] = mfma16(Rh, Kl, acc[rt][q]);
          }
        }
      }
    }
  };

  if (T0 < T1) {
    // tiles past the end are clamped to the last one: loaded and stored but never computed
    auto tc = [&](int64_t T) { return T < T1 ? T : T1 - 1; };
    Stage s0 = gload(T0);
    sstore(s0, 0);
    Stage s1 = gload(tc(T0 + 1));
    __syncthreads();
    int64_t T = T0;
    // pairs of tiles: on entry LDS buffer 0 holds tile T and s1 holds tile T + 1
    // the empty asm statements keep each prefetch issued before the compute it overlaps
    // (otherwise the scheduler may sink the loads below the LDS reads of the compute)
    for (; T + 1 < T1; T += 2) {
      s0 = gload(tc(T + 2));
      asm volatile("" ::: "memory");
      compute(0);
      sstore(s1, 1);
      __syncthreads();
      s1 = gload(tc(T + 3));
      asm volatile("" ::: "memory");
      compute(1);
      sstore(s0, 0);
      __syncthreads();
    }
    if (T < T1) compute(0);  // odd count: the last tile is in buffer 0
  }
  kz_deferred();  // the last tile's K Z products

  // write partial sums
  if constexpr (MODE == MODE_F32V) {
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) {
#pragma unroll
      for (int c = 0; c < NQ; ++c) {
        float v = accv[rt][c];
        v += __shfl_xor(v, 16);
        v += __shfl_xor(v, 32);
        const int64_t row = row_base + rt * 16 + lane % 16;
        if (lane < 16 && row < a.m && c < a.k) out[(row - out_row0) * a.k + c] = v;
      }
    }
  } else {
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) {
      const int64_t row = row_base + rt * 16 + lane % 16;
      if (row >= a.m) continue;
#pragma unroll
      for (int q = 0; q < NQ; ++q)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int rhs = q * 16 + 4 * (lane / 16) + j;
          if (rhs < a.k) out[(row - out_row0) * a.k + rhs] = acc[rt][q][j];
        }
    }
  }
}

template <int KS, int KERN, int MODE, int NQ, int RT>
__global__ __launch_bounds__(256, (mk_occupancy<KERN, MODE, NQ>())) void mk_kernel(MkArgs a) {
  __shared__ __attribute__((aligned(16))) char lds[2 * MkShape<KS, MODE, NQ>::BUF_BYTES];
  const int bid = blockIdx.x;
  const int prob = blockIdx.y;
  int split, rw;
  if (a.xcd_map) {
    // workgroups are dealt round-robin to the 8 XCDs: XCD x runs items
    // [x * grid/8, (x+1) * grid/8) of the split-major order, so the row workgroups of one
    // column split sit on one or two XCDs and share the split's column stream in their L2
    const int per = (int)gridDim.x / 8;
    const int item = (bid % 8) * per + bid / 8;
    split = item / a.rwg;
    rw = item % a.rwg;
  } else {
    split = bid / a.rwg;
    rw = bid % a.rwg;
  }
  const int64_t T0 = (int64_t)split * a.tiles_per_split;
  int64_t T1 = T0 + a.tiles_per_split;
  if (T1 > a.ntiles) T1 = a.ntiles;
  mk_tiles<KS, KERN, MODE, NQ, RT>(
      a, lds, a.colA + prob * a.bs_colA, static_cast<const char*>(a.rhs) + prob * a.bs_rhs,
      a.ridx ? a.ridx + prob * a.bs_ridx : nullptr, rw, T0, T1,
      a.part + prob * a.bs_part + (int64_t)split * a.m * a.k, 0);
}

// Wide tiles (MODE_F16W): the float16 mode on 32x32x16 MFMAs.  A wave takes two row tiles of
// 32 (64 rows, as the 16x16 form) against each column tile of 32.  The distance takes NS
// K-slices of 16 slots (NS = 3 for 3d + 6 <= 48, against 64 slots on 16x16x32), with the
// column fragments read from the same LDS tile in the 32x32 operand order (A[m][k] in lane
// m + 32 (k / 8), element k % 8) and the row fragments from the row vectors.  The K Z products
// are software-pipelined by one tile as in the 16x16 form; each accumulator adds the tiles
// in order.
template <int KS, int NS, int KERN, int NQW>
__device__ void mkw_tiles(const MkArgs& a, char* lds, const half8* colA_p, const void* rhs_p,
                          const int64_t* ridx, int rw, int64_t T0, int64_t T1, float* out) {
  constexpr int A_FR = 2 * KS * 64, R_FR = NQW * 2 * 64, TOTAL16 = A_FR + R_FR;
  constexpr int BUF_BYTES = ((TOTAL16 + 255) / 256) * 256 * 16;
  constexpr int LOADS16 = (TOTAL16 + 255) / 256;
  static_assert(NS >= 1 && NS <= 2 * KS, "K-slices within the packed slots");
  static_assert(LOADS16 <= 5, "tile loads per thread");
  const int tid = threadIdx.x;
  const int lane = tid % 64;
  const int wave = tid / 64;
  const int g = lane / 32;
  const int64_t row_base = ((int64_t)rw * WAVES + wave) * 64;
  // row fragments (B operand: B[k][n] in lane n + 32 (k / 8), element k % 8)
  half8 Bfr[2][NS];
  static_for<2>([&](auto rc) {
    constexpr int rt = decltype(rc)::value;
    const int64_t row = row_base + rt * 32 + lane % 32;
    const int64_t pt = row < a.m ? (ridx ? ridx[row] : row) : (ridx ? ridx[0] : 0);
    static_for<NS>([&](auto sc) {
      constexpr int sl = decltype(sc)::value;
      Bfr[rt][sl] = a.rowv[pt * 8 + 2 * sl + g];
    });
  });
#pragma unroll
  for (int rt = 0; rt < 2; ++rt)
#pragma unroll
    for (int sl = 0; sl < NS; ++sl) asm volatile("" ::"v"(Bfr[rt][sl]));
  // LDS positions of this lane's column fragments: column c = lane % 32, slots 16 s + 8 g..,
  // stored as [column half][K-step of 32][slot group of 8][16 columns]
  int aidx[NS];
  {
    const int c = lane % 32;
    static_for<NS>([&](auto sc) {
      constexpr int sl = decltype(sc)::value;
      const int hb = 2 * sl + g;
      aidx[sl] = ((c / 16) * KS + hb / 4) * 64 + (hb % 4) * 16 + c % 16;
    });
  }
  f16v acc[2][NQW];
  half8 Kp[2][2];
  half8 Rp[NQW][2];
  static_for<2>([&](auto rc) {
    constexpr int rt = decltype(rc)::value;
    static_for<NQW>([&](auto qc) {
      constexpr int q = decltype(qc)::value;
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[rt][q][r] = 0.0f;
    });
  });
  static_for<2>([&](auto ic) {
    constexpr int i = decltype(ic)::value;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      Kp[i][0][j] = (_Float16)0.0f;
      Kp[i][1][j] = (_Float16)0.0f;
    }
  });
  static_for<NQW>([&](auto qc) {
    constexpr int q = decltype(qc)::value;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      Rp[q][0][j] = (_Float16)0.0f;
      Rp[q][1][j] = (_Float16)0.0f;
    }
  });

  struct Stage {
    uint4 w0, w1, w2, w3, w4;
  };
  auto word = [](Stage& st, auto uc) __attribute__((always_inline)) -> uint4& {
    constexpr int u = decltype(uc)::value;
    if constexpr (u == 0) return st.w0;
    else if constexpr (u == 1) return st.w1;
    else if constexpr (u == 2) return st.w2;
    else if constexpr (u == 3) return st.w3;
    else return st.w4;
  };
  auto gload = [&](int64_t T) __attribute__((always_inline)) -> Stage {
    Stage st;
    const uint4* ca = reinterpret_cast<const uint4*>(colA_p) + T * A_FR;
    const uint4* rb = reinterpret_cast<const uint4*>(rhs_p) + T * R_FR;
    static_for<LOADS16>([&](auto uc) {
      constexpr int u = decltype(uc)::value;
      const int e = tid + u * 256;
      const uint4* src = e < A_FR ? ca + e : (e < TOTAL16 ? rb + (e - A_FR) : ca);
      word(st, uc) = *src;
    });
    return st;
  };
  auto sstore = [&](Stage st, int buf) __attribute__((always_inline)) {
    uint4* dst = reinterpret_cast<uint4*>(lds + buf * BUF_BYTES);
    static_for<LOADS16>([&](auto uc) {
      constexpr int u = decltype(uc)::value;
      dst[tid + u * 256] = word(st, uc);
    });
  };
  auto kz_deferred = [&]() __attribute__((always_inline)) {
    static_for<2>([&](auto rc) {
      constexpr int rt = decltype(rc)::value;
      static_for<NQW>([&](auto qc) {
        constexpr int q = decltype(qc)::value;
        acc[rt][q] = mfma32(Rp[q][0], Kp[rt][0], acc[rt][q]);
        acc[rt][q] = mfma32(Rp[q][1], Kp[rt][1], acc[rt][q]);
      });
    });
  };
  auto compute = [&](int buf) __attribute__((always_inline)) {
    const half8* Af = reinterpret_cast<const half8*>(lds + buf * BUF_BYTES);
    kz_deferred();
    const half8* Rf = Af + A_FR;
    static_for<NQW>([&](auto qc) {
      constexpr int q = decltype(qc)::value;
      Rp[q][0] = Rf[(q * 2 + 0) * 64 + lane];
      Rp[q][1] = Rf[(q * 2 + 1) * 64 + lane];
    });
    half8 A[NS];
    static_for<NS>([&](auto sc) {
      constexpr int sl = decltype(sc)::value;
      A[sl] = Af[aidx[sl]];
    });
    static_for<2>([&](auto rc) {
      constexpr int rt = decltype(rc)::value;
      f16v D;
#pragma unroll
      for (int r = 0; r < 16; ++r) D[r] = 0.0f;
      static_for<NS>([&](auto sc) {
        constexpr int sl = decltype(sc)::value;
        D = mfma32(A[sl], Bfr[rt][sl], D);
      });
      static_for<2>([&](auto tc) {
        constexpr int t = decltype(tc)::value;
        half8 Kh;
#pragma unroll
        for (int j = 0; j < 8; ++j) Kh[j] = (_Float16)kval<KERN>(D[8 * t + j], a.p);
        Kp[rt][t] = Kh;
      });
    });
  };

  if (T0 < T1) {
    auto tc = [&](int64_t T) { return T < T1 ? T : T1 - 1; };
    Stage s0 = gload(T0);
    sstore(s0, 0);
    Stage s1 = gload(tc(T0 + 1));
    __syncthreads();
    int64_t T = T0;
    for (; T + 1 < T1; T += 2) {
      s0 = gload(tc(T + 2));
      asm volatile("" ::: "memory");
      compute(0);
      sstore(s1, 1);
      __syncthreads();
      s1 = gload(tc(T + 3));
      asm volatile("" ::: "memory");
      compute(1);
      sstore(s0, 0);
      __syncthreads();
    }
    if (T < T1) compute(0);
  }
  kz_deferred();

  // partial sums: lane l, register r is right-hand side 32 q + 8 (r / 4) + 4 g + r % 4 of
  // row 32 rt + l % 32
  static_for<2>([&](auto rc) {
    constexpr int rt = decltype(rc)::value;
    const int64_t row = row_base + rt * 32 + lane % 32;
    if (row < a.m) {
      static_for<NQW>([&](auto qc) {
        constexpr int q = decltype(qc)::value;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int rhs = q * 32 + 8 * (r / 4) + 4 * g + r % 4;
          if (rhs < a.k) out[row * a.k + rhs] = acc[rt][q][r];
        }
      });
    }
  });
}

template <int KS, int NS, int KERN, int NQW>
__global__ __launch_bounds__(256, 2) void mkw_kernel(MkArgs a) {
  constexpr int TOTAL16 = 2 * KS * 64 + NQW * 2 * 64;
  __shared__ __attribute__((aligned(16))) char lds[2 * ((TOTAL16 + 255) / 256) * 256 * 16];
  const int bid = blockIdx.x;
  const int prob = blockIdx.y;
  int split, rw;
  if (a.xcd_map) {
    const int per = (int)gridDim.x / 8;
    const int item = (bid % 8) * per + bid / 8;
    split = item / a.rwg;
    rw = item % a.rwg;
  } else {
    split = bid / a.rwg;
    rw = bid % a.rwg;
  }
  const int64_t T0 = (int64_t)split * a.tiles_per_split;
  int64_t T1 = T0 + a.tiles_per_split;
  if (T1 > a.ntiles) T1 = a.ntiles;
  mkw_tiles<KS, NS, KERN, NQW>(
      a, lds, a.colA + prob * a.bs_colA, static_cast<const char*>(a.rhs) + prob * a.bs_rhs,
      a.ridx ? a.ridx + prob * a.bs_ridx : nullptr, rw, T0, T1,
      a.part + prob * a.bs_part + (int64_t)split * a.m * a.k);
}

// Wide tiles for the float32 vector mode (MODE_F32V, one to four right-hand sides): the
// distances on 32x32x16 MFMAs as in the wide float16 form (NS K-slices of 16 of the packed
// slots, 3d + 6 <= 48 for d <= 14, against 64 slots in two K-steps of the 16x16x32 form),
// the kernel values and K Z in float32 on the vector ALUs.  A wave takes two row tiles of 32
// (64 rows); lane l holds row l % 32 of each and the 16 columns 8 (r / 4) + 4 g + r % 4 of
// the tile (g = l / 32), whose right-hand-side values it reads as four runs of four columns.
// The two halves of a row's columns are added across lanes 32 apart after the last tile.
template <int KS, int NS, int KERN, int KC>
__device__ void mkv_tiles(const MkArgs& a, char* lds, const half8* colA_p, const void* rhs_p,
                          const int64_t* ridx, int rw, int64_t T0, int64_t T1, float* out) {
  constexpr int A_FR = 2 * KS * 64, R_W = (TILE * KC * 4) / 16, TOTAL16 = A_FR + R_W;
  constexpr int BUF_BYTES = ((TOTAL16 + 255) / 256) * 256 * 16;
  constexpr int LOADS16 = (TOTAL16 + 255) / 256;
  static_assert(NS >= 1 && NS <= 2 * KS, "K-slices within the packed slots");
  static_assert(LOADS16 <= 5, "tile loads per thread");
  const int tid = threadIdx.x;
  const int lane = tid % 64;
  const int wave = tid / 64;
  const int g = lane / 32;
  const int64_t row_base = ((int64_t)rw * WAVES + wave) * 64;
  half8 Bfr[2][NS];
  static_for<2>([&](auto rc) {
    constexpr int rt = decltype(rc)::value;
    const int64_t row = row_base + rt * 32 + lane % 32;
    const int64_t pt = row < a.m ? (ridx ? ridx[row] : row) : (ridx ? ridx[0] : 0);
    static_for<NS>([&](auto sc) {
      constexpr int sl = decltype(sc)::value;
      Bfr[rt][sl] = a.rowv[pt * 8 + 2 * sl + g];
    });
  });
#pragma unroll
  for (int rt = 0; rt < 2; ++rt)
#pragma unroll
    for (int sl = 0; sl < NS; ++sl) asm volatile("" ::"v"(Bfr[rt][sl]));
  int aidx[NS];
  {
    const int c = lane % 32;
    static_for<NS>([&](auto sc) {
      constexpr int sl = decltype(sc)::value;
      const int hb = 2 * sl + g;
      aidx[sl] = ((c / 16) * KS + hb / 4) * 64 + (hb % 4) * 16 + c % 16;
    });
  }
  float acc[2][KC];
#pragma unroll
  for (int rt = 0; rt < 2; ++rt)
#pragma unroll
    for (int c = 0; c < KC; ++c) acc[rt][c] = 0.0f;

  struct Stage {
    uint4 w0, w1, w2, w3, w4;
  };
  auto word = [](Stage& st, auto uc) __attribute__((always_inline)) -> uint4& {
    constexpr int u = decltype(uc)::value;
    if constexpr (u == 0) return st.w0;
    else if constexpr (u == 1) return st.w1;
    else if constexpr (u == 2) return st.w2;
    else if constexpr (u == 3) return st.w3;
    else return st.w4;
  };
  auto gload = [&](int64_t T) __attribute__((always_inline)) -> Stage {
    Stage st;
    const uint4* ca = reinterpret_cast<const uint4*>(colA_p) + T * A_FR;
    const uint4* rb = reinterpret_cast<const uint4*>(rhs_p) + T * R_W;
    static_for<LOADS16>([&](auto uc) {
      constexpr int u = decltype(uc)::value;
      const int e = tid + u * 256;
      const uint4* src = e < A_FR ? ca + e : (e < TOTAL16 ? rb + (e - A_FR) : ca);
      word(st, uc) = *src;
    });
    return st;
  };
  auto sstore = [&](Stage st, int buf) __attribute__((always_inline)) {
    uint4* dst = reinterpret_cast<uint4*>(lds + buf * BUF_BYTES);
    static_for<LOADS16>([&](auto uc) {
      constexpr int u = decltype(uc)::value;
      dst[tid + u * 256] = word(st, uc);
    });
  };
  auto compute = [&](int buf) __attribute__((always_inline)) {
    const half8* Af = reinterpret_cast<const half8*>(lds + buf * BUF_BYTES);
    const float* zr = reinterpret_cast<const float*>(Af + A_FR);
    half8 A[NS];
    static_for<NS>([&](auto sc) {
      constexpr int sl = decltype(sc)::value;
      A[sl] = Af[aidx[sl]];
    });
    // right-hand-side values of this lane's 16 columns: zc[r][c] for column 8 (r / 4) + 4 g + r % 4
    float zc[16][KC];
    static_for<4>([&](auto qc) {
      constexpr int q = decltype(qc)::value;
      const float4* zp = reinterpret_cast<const float4*>(zr + (8 * q + 4 * g) * KC);
      static_for<KC>([&](auto wc) {
        constexpr int w = decltype(wc)::value;
        const float4 v = zp[w];
        const float f[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int flat = 4 * w + e;  // (column within the run) * KC + right-hand side
          zc[4 * q + flat / KC][flat % KC] = f[e];
        }
      });
    });
    // both row tiles' distances first, so that row tile 1's MFMAs run beside row tile 0's
    // kernel values; all 16 values of a row tile before their products (independent chains)
    f16v D[2];
    static_for<2>([&](auto rc) {
      constexpr int rt = decltype(rc)::value;
#pragma unroll
      for (int r = 0; r < 16; ++r) D[rt][r] = 0.0f;
      static_for<NS>([&](auto sc) {
        constexpr int sl = decltype(sc)::value;
        D[rt] = mfma32(A[sl], Bfr[rt][sl], D[rt]);
      });
    });
    if constexpr (KC == 1 && (KERN == ADASAP_MATERN32 || KERN == ADASAP_MATERN52)) {
      // One right-hand side: the Matern polynomial is folded into the product.  With
      // u = a log2(e) (a = p r / ell) and e = 2^-u, k z = e (1 + a) z = e (z + u (ln2 z)) for
      // 3/2 and e (z + u (ln2 z + u (ln2^2 / 3) z)) for 5/2; the column factors are formed
      // once per tile, so a pair costs the two transcendentals, one multiply and two or three
      // fmas instead of the polynomial's multiplies and adds and the product's fma.
      constexpr float LN2 = 0.6931471805599453f;
      float z1[16], z2[16];
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        z1[r] = LN2 * zc[r][0];
        z2[r] = (LN2 * LN2 / 3.0f) * zc[r][0];
      }
      const float pl = a.p * 1.4426950408889634f;
      static_for<2>([&](auto rc) {
        constexpr int rt = decltype(rc)::value;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          // the hardware square root of |s| as in kval
          const float u = __builtin_amdgcn_sqrtf(__builtin_fabsf(D[rt][r])) * pl;
          const float e = __builtin_amdgcn_exp2f(-u);
          float t;
          if constexpr (KERN == ADASAP_MATERN32) t = __builtin_fmaf(u, z1[r], zc[r][0]);
          else t = __builtin_fmaf(u, __builtin_fmaf(u, z2[r], z1[r]), zc[r][0]);
          acc[rt][0] = __builtin_fmaf(e, t, acc[rt][0]);
        }
      });
    } else {
      static_for<2>([&](auto rc) {
        constexpr int rt = decltype(rc)::value;
        float kv[16];
#pragma unroll
        for (int r = 0; r < 16; ++r) kv[r] = kval<KERN>(D[rt][r], a.p);
#pragma unroll
        for (int r = 0; r < 16; ++r)
#pragma unroll
          for (int c = 0; c < KC; ++c) acc[rt][c] = __builtin_fmaf(kv[r], zc[r][c], acc[rt][c]);
      });
    }
  };

  if (T0 < T1) {
    auto tc = [&](int64_t T) { return T < T1 ? T : T1 - 1; };
    Stage s0 = gload(T0);
    sstore(s0, 0);
    Stage s1 = gload(tc(T0 + 1));
    __syncthreads();
    int64_t T = T0;
    for (; T + 1 < T1; T += 2) {
      s0 = gload(tc(T + 2));
      asm volatile("" ::: "memory");
      compute(0);
      sstore(s1, 1);
      __syncthreads();
      s1 = gload(tc(T + 3));
      asm volatile("" ::: "memory");
      compute(1);
      sstore(s0, 0);
      __syncthreads();
    }
    if (T < T1) compute(0);
  }
  static_for<2>([&](auto rc) {
    constexpr int rt = decltype(rc)::value;
    const int64_t row = row_base + rt * 32 + lane % 32;
#pragma unroll
    for (int c = 0; c < KC; ++c) {
      const float v = acc[rt][c] + __shfl_xor(acc[rt][c], 32);
      if (g == 0 && row < a.m && c < a.k) out[row * a.k + c] = v;
    }
  });
}

template <int KS, int NS, int KERN, int KC>
__global__ __launch_bounds__(256, 4) void mkv_kernel(MkArgs a) {
  constexpr int TOTAL16 = 2 * KS * 64 + (TILE * KC * 4) / 16;
  __shared__ __attribute__((aligned(16))) char lds[2 * ((TOTAL16 + 255) / 256) * 256 * 16];
  const int bid = blockIdx.x;
  const int prob = blockIdx.y;
  int split, rw;
  if (a.xcd_map) {
    const int per = (int)gridDim.x / 8;
    const int item = (bid % 8) * per + bid / 8;
    split = item / a.rwg;
    rw = item % a.rwg;
  } else {
    split = bid / a.rwg;
    rw = bid % a.rwg;
  }
  const int64_t T0 = (int64_t)split * a.tiles_per_split;
  int64_t T1 = T0 + a.tiles_per_split;
  if (T1 > a.ntiles) T1 = a.ntiles;
  mkv_tiles<KS, NS, KERN, KC>(
      a, lds, a.colA + prob * a.bs_colA, static_cast<const char*>(a.rhs) + prob * a.bs_rhs,
      a.ridx ? a.ridx + prob * a.bs_ridx : nullptr, rw, T0, T1,
      a.part + prob * a.bs_part + (int64_t)split * a.m * a.k);
}

// Persistent work-queue form for a batch of problems with uneven column counts: each
// workgroup takes (problem, row workgroup, tile range) items from its XCD's counter until that
// XCD's range of the table is exhausted; an item writes its partial sums to
// part[slot][rows of its workgroup][k].  Workgroups are placed on the XCDs round-robin, so
// blockIdx.x % 8 names the XCD, and the items of one tile range (its row workgroups, adjacent
// in the range) meet in that XCD's L2.  Every range has drainers once the grid holds 8
// workgroups; the placement only decides locality, not which items run.
template <int KS, int KERN, int MODE, int NQ, int RT>
__global__ __launch_bounds__(256, (mk_occupancy<KERN, MODE, NQ>())) void mkq_kernel(MkArgs a) {
  __shared__ __attribute__((aligned(16))) char lds[2 * MkShape<KS, MODE, NQ>::BUF_BYTES];
  __shared__ int s_item;
  constexpr int ROWS = WAVES * RT * 16;
  const int x = (int)(blockIdx.x % QXCDS);
  const int beg = a.qbeg[x], end = a.qbeg[x + 1];
  for (;;) {
    if (threadIdx.x == 0) s_item = beg + atomicAdd(a.counter + x * QCOUNTER_STRIDE, 1);
    __syncthreads();
    const int item = s_item;
    __syncthreads();
    if (item >= end) break;
    const MkItem it = a.items[item];
    mk_tiles<KS, KERN, MODE, NQ, RT>(
        a, lds, a.colA + a.colA_off[it.prob],
        static_cast<const char*>(a.rhs) + a.rhs_off[it.prob],
        a.ridx + (int64_t)it.prob * a.bs_ridx, it.rw, it.T0, it.T1,
        a.part + (int64_t)it.slot * ROWS * a.k, (int64_t)it.rw * ROWS);
  }
}

// out[i, c] = scale[c] * sum_s part[s, i, c] + epilogue
__global__ void mk_reduce_kernel(const float* __restrict__ part, int splits, int64_t m, int k,
                                 const float* __restrict__ scale, KbEpilogue ep,
                                 void* __restrict__ out, DT ot) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= m * k) return;
  {
    // batch: problem blockIdx.y
    const int64_t pb = blockIdx.y;
    part += pb * splits * m * k;
    if (scale) scale += pb * k;
    out = static_cast<char*>(out) + pb * m * k * (ot == DT::F64 ? 8 : 4);
    if (ep.E1) ep.E1 = static_cast<const char*>(ep.E1) + pb * ep.bsE1 * (ep.e1t == DT::F64 ? 8 : 4);
    if (ep.E2) ep.E2 = static_cast<const char*>(ep.E2) + pb * ep.bsE2 * (ep.e2t == DT::F64 ? 8 : 4);
    if (ep.e1idx) ep.e1idx += pb * ep.bsIdx;
    if (ep.e2idx) ep.e2idx += pb * ep.bsIdx;
  }
  const int64_t i = e / k;
  const int c = (int)(e % k);
  double s = 0.0;
  // (the loads of eight splits are issued together; the sum keeps the split order)
#pragma unroll 8
  for (int sp = 0; sp < splits; ++sp) s += (double)part[((int64_t)sp * m + i) * k + c];
  if (scale) s *= (double)scale[c];
  s *= ep.kscale;
  auto ld = [](const void* p, DT t, int64_t j) {
    return t == DT::F64 ? static_cast<const double*>(p)[j] : (double)static_cast<const float*>(p)[j];
  };
  if (ep.E1) s += ep.a1 * ld(ep.E1, ep.e1t, (ep.e1idx ? ep.e1idx[i] : i) * ep.lde1 + c);
  if (ep.E2) s += ep.a2 * ld(ep.E2, ep.e2t, (ep.e2idx ? ep.e2idx[i] : i) * ep.lde2 + c);
  if (ot == DT::F64) static_cast<double*>(out)[e] = s;
  else static_cast<float*>(out)[e] = (float)s;
}

// ---------------------------------------------------------------- dispatch
template <int KS, int KERN, int MODE, int NQ, int RT>
void launch_mk(const MkArgs& a, int grid, hipStream_t s) {
  hipLaunchKernelGGL((mk_kernel<KS, KERN, MODE, NQ, RT>), dim3(grid), dim3(256), 0, s, a);
}

template <int KS, int KERN, int MODE>
adasap_status_t disp_nq(const MkArgs& a, int nq, int grid, hipStream_t s) {
  constexpr int R4 = rt_of(MODE, 4);
  switch (nq) {
    case 1: launch_mk<KS, KERN, MODE, 1, R4>(a, grid, s); break;
    case 2: launch_mk<KS, KERN, MODE, 2, R4>(a, grid, s); break;
    case 3: launch_mk<KS, KERN, MODE, 3, R4>(a, grid, s); break;
    case 4: launch_mk<KS, KERN, MODE, 4, R4>(a, grid, s); break;
    case 5: launch_mk<KS, KERN, MODE, 5, 2>(a, grid, s); break;
    case 6: launch_mk<KS, KERN, MODE, 6, 2>(a, grid, s); break;
    case 7: launch_mk<KS, KERN, MODE, 7, 2>(a, grid, s); break;
    default: launch_mk<KS, KERN, MODE, 8, 2>(a, grid, s); break;
  }
  return ADASAP_OK;
}

template <int KS, int KERN>
adasap_status_t disp_mode(const MkArgs& a, int mode, int nq, int grid, hipStream_t s) {
  if (mode == MODE_F16) return disp_nq<KS, KERN, MODE_F16>(a, nq, grid, s);
  if (mode == MODE_F16X3) return disp_nq<KS, KERN, MODE_F16X3>(a, nq, grid, s);
  set_error("internal: the float32 vector mode runs the wide-tile kernel");
  return ADASAP_ERR_INVALID_ARG;
}

template <int KS>
adasap_status_t disp_kern(const MkArgs& a, int kern, int mode, int nq, int grid, hipStream_t s) {
  switch (kern) {
    case ADASAP_RBF: return disp_mode<KS, ADASAP_RBF>(a, mode, nq, grid, s);
    case ADASAP_MATERN12: return disp_mode<KS, ADASAP_MATERN12>(a, mode, nq, grid, s);
    case ADASAP_MATERN32: return disp_mode<KS, ADASAP_MATERN32>(a, mode, nq, grid, s);
    default: return disp_mode<KS, ADASAP_MATERN52>(a, mode, nq, grid, s);
  }
}

template <int KS, int KERN, int MODE, int NQ, int RT>
void launch_mk_grid(const MkArgs& a, dim3 grid, hipStream_t s) {
  hipLaunchKernelGGL((mk_kernel<KS, KERN, MODE, NQ, RT>), grid, dim3(256), 0, s, a);
}

template <int KS, int KERN>
void disp_mode_grid(const MkArgs& a, int mode, int nq, dim3 grid, hipStream_t s) {
  if (mode == MODE_F16X3) {
    switch (nq) {
      case 1: launch_mk_grid<KS, KERN, MODE_F16X3, 1, 4>(a, grid, s); break;
      case 2: launch_mk_grid<KS, KERN, MODE_F16X3, 2, 4>(a, grid, s); break;
      case 3: launch_mk_grid<KS, KERN, MODE_F16X3, 3, 4>(a, grid, s); break;
      case 4: launch_mk_grid<KS, KERN, MODE_F16X3, 4, 4>(a, grid, s); break;
      case 5: launch_mk_grid<KS, KERN, MODE_F16X3, 5, 2>(a, grid, s); break;
      case 6: launch_mk_grid<KS, KERN, MODE_F16X3, 6, 2>(a, grid, s); break;
      case 7: launch_mk_grid<KS, KERN, MODE_F16X3, 7, 2>(a, grid, s); break;
      default: launch_mk_grid<KS, KERN, MODE_F16X3, 8, 2>(a, grid, s); break;
    }
  }
}

template <int KS, int NS, int KERN>
void launch_wide(const MkArgs& a, int nqw, int grid, hipStream_t s) {
  if (nqw == 1) hipLaunchKernelGGL((mkw_kernel<KS, NS, KERN, 1>), dim3(grid), dim3(256), 0, s, a);
  else hipLaunchKernelGGL((mkw_kernel<KS, NS, KERN, 2>), dim3(grid), dim3(256), 0, s, a);
}

template <int KS, int NS>
void launch_wide_kern(const MkArgs& a, int kern, int nqw, int grid, hipStream_t s) {
  switch (kern) {
    case ADASAP_RBF: launch_wide<KS, NS, ADASAP_RBF>(a, nqw, grid, s); break;
    case ADASAP_MATERN12: launch_wide<KS, NS, ADASAP_MATERN12>(a, nqw, grid, s); break;
    case ADASAP_MATERN32: launch_wide<KS, NS, ADASAP_MATERN32>(a, nqw, grid, s); break;
    default: launch_wide<KS, NS, ADASAP_MATERN52>(a, nqw, grid, s); break;
  }
}

adasap_status_t disp_wide(const MkArgs& a, int ks, int ns, int kern, int nqw, int grid,
                          hipStream_t s) {
  if (ks == 1) launch_wide_kern<1, 2>(a, kern, nqw, grid, s);
  else if (ns == 3) launch_wide_kern<2, 3>(a, kern, nqw, grid, s);
  else launch_wide_kern<2, 4>(a, kern, nqw, grid, s);
  return ADASAP_OK;
}

template <int KS, int NS, int KERN>
void launch_vwide(const MkArgs& a, int kc, dim3 grid, hipStream_t s) {
  if (kc == 1) hipLaunchKernelGGL((mkv_kernel<KS, NS, KERN, 1>), grid, dim3(256), 0, s, a);
  else if (kc == 2) hipLaunchKernelGGL((mkv_kernel<KS, NS, KERN, 2>), grid, dim3(256), 0, s, a);
  else hipLaunchKernelGGL((mkv_kernel<KS, NS, KERN, 4>), grid, dim3(256), 0, s, a);
}

template <int KS, int NS>
void launch_vwide_kern(const MkArgs& a, int kern, int kc, dim3 grid, hipStream_t s) {
  switch (kern) {
    case ADASAP_RBF: launch_vwide<KS, NS, ADASAP_RBF>(a, kc, grid, s); break;
    case ADASAP_MATERN12: launch_vwide<KS, NS, ADASAP_MATERN12>(a, kc, grid, s); break;
    case ADASAP_MATERN32: launch_vwide<KS, NS, ADASAP_MATERN32>(a, kc, grid, s); break;
    default: launch_vwide<KS, NS, ADASAP_MATERN52>(a, kc, grid, s); break;
  }
}

adasap_status_t disp_vwide(const MkArgs& a, int ks, int ns, int kern, int kc, dim3 grid,
                           hipStream_t s) {
  if (ks == 1) launch_vwide_kern<1, 2>(a, kern, kc, grid, s);
  else if (ns == 3) launch_vwide_kern<2, 3>(a, kern, kc, grid, s);
  else launch_vwide_kern<2, 4>(a, kern, kc, grid, s);
  return ADASAP_OK;
}

inline int ksteps(int d) { return 3 * d + 6 <= 32 ? 1 : 2; }

double sigma_for(int kern, double ell) {
  return kern == ADASAP_RBF ? std::sqrt(LOG2E) / ell : std::sqrt(2.0) / ell;
}

float matern_factor(int kern) {
  return kern == ADASAP_MATERN12 ? 1.0f : (kern == ADASAP_MATERN32 ? 1.7320508075688772f : 2.23606797749979f);
}

struct RhsDesc {
  int mode;     // MODE_*
  int nq;       // 16-column tiles (F16 modes) or KC (F32V)
  const void* p;
  const float* scale;  // null for F32V
};

// the product: rows (ridx into rowv, or rowv itself) x column fragments, into out (+ epilogue)
adasap_status_t mk_run(const half8* colA, int64_t ntiles, const half8* rowv,
                       const int64_t* ridx, int64_t m, int d, int kern, const RhsDesc& rd, int k,
                       void* out, DT ot, const KbEpilogue& ep, DevBuf& part, hipStream_t s,
                       hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr, int ks_force = 0,
                       int cap_cus = 0) {
  if (m <= 0) return ADASAP_OK;
  const int RT = rt_of(rd.mode, rd.nq);
  const int rows_per_wg = WAVES * RT * 16;
  const int rwg = (int)((m + rows_per_wg - 1) / rows_per_wg);
  int splits;
  // cap_cus > 0: one resident round on 7/8 of two workgroup slots per CU (three for the
  // float32 vector mode, whose 128-VGPR workgroups leave a SIMD 128 registers beside three of
  // them), for products of up to 64 row workgroups (longer products amortise the concurrent
  // stream's work anyway), and only if the capped grid fills at least 9/10 of the cap.
  // Measured at the vector mode: 7/8 of four slots per CU, or all of three, leaves the second
  // stream's kernels too little room and the iteration is slower.
  int wg_cap = 0;
  if (cap_cus > 0 && rwg <= 64) {
    const int slots = cap_cus * (rd.mode == MODE_F32V ? 3 : 2);
    wg_cap = slots - slots / 8;
    if ((wg_cap / rwg) * rwg * 10 < wg_cap * 9) wg_cap = 0;
  }
  if (wg_cap > 0) {
    // one resident round that leaves some workgroup slots free for a concurrent stream
    splits = wg_cap / rwg;
    if (splits > ntiles) splits = (int)(ntiles > 0 ? ntiles : 1);
  } else {
    // aim for >= 2048 workgroups (8 per CU) when the column range allows it
    splits = (2048 + rwg - 1) / rwg;
    if (splits > ntiles) splits = (int)(ntiles > 0 ? ntiles : 1);
    if (splits >= 8) splits -= splits % 8;
  }
  if (splits < 1) splits = 1;
  int64_t tps = (ntiles + splits - 1) / splits;
  if (tps < 1) tps = 1;
  splits = (int)((ntiles + tps - 1) / tps);
  if (splits < 1) splits = 1;
  const int xcd_map = ((int64_t)rwg * splits % 8 == 0) ? 1 : 0;
  ADASAP_TRY(part.ensure((size_t)splits * m * k * sizeof(float)));
  MkArgs a{};
  a.colA = colA;
  a.rowv = rowv;
  a.ridx = ridx;
  a.m = m;
  a.rhs = rd.p;
  a.ntiles = ntiles;
  a.tiles_per_split = tps;
  a.splits = splits;
  a.rwg = rwg;
  a.xcd_map = xcd_map;
  a.part = part.as<float>();
  a.k = k;
  a.p = matern_factor(kern);
  const int grid = rwg * splits;
  const int KS = ks_force ? ks_force : ksteps(d);
  if (ev0) ADASAP_HIP(hipEventRecord(ev0, s));
  if (rd.mode == MODE_F16W) {
    // K-slices of 16 for the 3d + 6 distance slots: 2 (d <= 8), 3 (d <= 14) or 4
    const int ns = KS == 1 ? 2 : (3 * d + 6 <= 48 ? 3 : 4);
    ADASAP_TRY(disp_wide(a, KS, ns, kern, rd.nq, grid, s));
  } else if (rd.mode == MODE_F32V) {
    const int ns = KS == 1 ? 2 : (3 * d + 6 <= 48 ? 3 : 4);
    ADASAP_TRY(disp_vwide(a, KS, ns, kern, rd.nq, dim3(grid), s));
  } else if (KS == 1) {
    ADASAP_TRY(disp_kern<1>(a, kern, rd.mode, rd.nq, grid, s));
  } else {
    ADASAP_TRY(disp_kern<2>(a, kern, rd.mode, rd.nq, grid, s));
  }
  ADASAP_LAUNCH_CHECK();
  if (ev1) ADASAP_HIP(hipEventRecord(ev1, s));
  hipLaunchKernelGGL(mk_reduce_kernel, dim3((unsigned)((m * k + 255) / 256)), dim3(256), 0, s,
                     part.as<float>(), splits, m, k, rd.scale, ep, out, ot);
  ADASAP_LAUNCH_CHECK();
  return ADASAP_OK;
}

// pack a right-hand side R (rows x k, type rt, optional row gather idx) for ntiles column tiles
adasap_status_t pack_rhs(const void* R, DT rt, int64_t rows, int k, int64_t ldr,
                         const int64_t* idx, int64_t ntiles, int mode, DevBuf& buf,
                         DevBuf& scale, DevBuf& tmp, RhsDesc& rd, hipStream_t s) {
  rd.mode = mode;
  if (mode == MODE_F32V) {
    const int kc = k == 1 ? 1 : (k == 2 ? 2 : 4);
    const int64_t npad = ntiles * TILE;
    ADASAP_TRY(buf.ensure((size_t)npad * kc * sizeof(float)));
    const int64_t tot = npad * kc;
    if (kc == 1)
      hipLaunchKernelGGL(rhspack32_kernel<1>, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, R, rt, rows, k, ldr, idx, npad, buf.as<float>());
    else if (kc == 2)
      hipLaunchKernelGGL(rhspack32_kernel<2>, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, R, rt, rows, k, ldr, idx, npad, buf.as<float>());
    else
      hipLaunchKernelGGL(rhspack32_kernel<4>, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, R, rt, rows, k, ldr, idx, npad, buf.as<float>());
    ADASAP_LAUNCH_CHECK();
    rd.nq = kc;
    rd.p = buf.p;
    rd.scale = nullptr;
    return ADASAP_OK;
  }
  const bool wide = mode == MODE_F16W;
  // wide tiles: one or two blocks of 32 right-hand sides; otherwise tiles of 16
  const int nq = wide ? (k <= 32 ? 1 : 2) : (k + 15) / 16;
  const int parts = mode == MODE_F16X3 ? 2 : 1;
  ADASAP_TRY(buf.ensure((size_t)ntiles * nq * (wide ? 2 : parts) * 64 * 16));
  ADASAP_TRY(scale.ensure((size_t)k * sizeof(float)));
  // column maxima of the (gathered) right-hand side
  const int64_t rpb = colmax_rows_per_block(rows);
  const int nblk = (int)((rows + rpb - 1) / rpb);
  ADASAP_TRY(tmp.ensure((size_t)(nblk > 0 ? nblk : 1) * k * sizeof(float)));
  if (idx) {
    // gathered rows: maxima over all of R are a valid (larger or equal) bound
    set_error("internal: gathered float16 right-hand sides are packed from a contiguous copy");
    return ADASAP_ERR_INVALID_ARG;
  }
  if (nblk > 0) {
    hipLaunchKernelGGL(colmax_partial_kernel, dim3(nblk), dim3(256), 0, s, R, rt, rows, k, ldr,
                       tmp.as<float>(), rpb);
    ADASAP_LAUNCH_CHECK();
  }
  hipLaunchKernelGGL(colmax_final_kernel, dim3(k), dim3(256), 0, s, tmp.as<float>(), nblk, k,
                     scale.as<float>());
  ADASAP_LAUNCH_CHECK();
  if (wide) {
    const int64_t tot = ntiles * nq * 128;
    hipLaunchKernelGGL(rhspackw_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, R,
                       rt, rows, k, ldr, scale.as<float>(), ntiles, nq, buf.as<half8>());
  } else {
    const int64_t tot = ntiles * nq * 64;
    hipLaunchKernelGGL(rhspack16_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, R,
                       rt, rows, k, ldr, nullptr, scale.as<float>(), ntiles, nq, parts,
                       buf.as<half8>());
  }
  ADASAP_LAUNCH_CHECK();
  rd.nq = nq;
  rd.p = buf.p;
  rd.scale = scale.as<float>();
  return ADASAP_OK;
}

// ---------------------------------------------------------------- fused update and packing
// The Nesterov update of the MIXED path (Alg. NestAcc) and the float16 packing of the next
// iterate for Step I in one streaming pass.  Each workgroup takes tiles of 32 rows
// (grid-stride): it applies the all-rows 2x2 map to (V, Z), the block-row correction to the
// rows of B (found through pos: pos[i] = (stamp << 32) | j when row i is B[j] in the current
// iteration), writes V, Z and, when asked, W, and packs the new Z tile in the operand order of
// the Step-I product with the per-column power-of-two scales computed beforehand from a bound
// (fused_scale_kernel).  It also records per-column maxima of |V| and |Z| for the next bound.
constexpr int FU_TILES_MAX = 4096;  // workgroups of the fused pass (grid-stride over tiles)

__global__ __launch_bounds__(256) void vzmax_partial_kernel(int64_t n, int k, int64_t ntiles,
                                                            const float* __restrict__ V,
                                                            const float* __restrict__ Z,
                                                            float* __restrict__ part) {
  __shared__ unsigned int mv[128], mz[128];
  for (int c = threadIdx.x; c < k; c += 256) mv[c] = mz[c] = 0u;
  __syncthreads();
  for (int64_t T = blockIdx.x; T < ntiles; T += gridDim.x) {
    for (int e = threadIdx.x; e < 32 * k; e += 256) {
      const int64_t i = T * TILE + e / k;
      const int c = e % k;
      if (i < n) {
        atomicMax(&mv[c], __float_as_uint(fabsf(V[i * k + c])));
        atomicMax(&mz[c], __float_as_uint(fabsf(Z[i * k + c])));
      }
    }
  }
  __syncthreads();
  for (int c = threadIdx.x; c < k; c += 256) {
    part[((int64_t)blockIdx.x * 2 + 0) * k + c] = __uint_as_float(mv[c]);
    part[((int64_t)blockIdx.x * 2 + 1) * k + c] = __uint_as_float(mz[c]);
  }
}

__global__ void pos_scatter_kernel(int64_t b, const int64_t* __restrict__ B, uint32_t stamp,
                                   int64_t* __restrict__ pos) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j < b) pos[B[j]] = (int64_t)(((uint64_t)stamp << 32) | (uint64_t)j);
}

// scale[c]: power of two with bound_c / scale <= 2^14, bound_c = max(|V|, |Z|) over the previous
// state (partials) + coef * eta * max_j |D[j, c]| (a bound on the new |Z|: the all-rows map is a
// convex combination, the block correction adds at most coef * eta * |D|)
__global__ __launch_bounds__(256) void fused_scale_kernel(int nwg, int k, const float* __restrict__ part,
                                                          int dblk, const float* __restrict__ dpart,
                                                          const IterScalars* __restrict__ sc,
                                                          double coef, float* __restrict__ scale) {
  __shared__ double red[256];
  const int c = blockIdx.x;
  double m = 0.0;
  for (int w = threadIdx.x; w < nwg; w += 256) {
    const double a = part[((int64_t)w * 2 + 0) * k + c], z = part[((int64_t)w * 2 + 1) * k + c];
    m = fmax(m, fmax(a, z));
  }
  // max |D| of the column from the per-block maxima (colmax_partial_kernel: a float bound of
  // each block's maximum, rounded to nearest; a maximum rounded down by an ulp leaves the
  // power-of-two scale's factor-4 headroom below the float16 range)
  double dm = 0.0;
  for (int j = threadIdx.x; j < dblk; j += 256) dm = fmax(dm, (double)dpart[(int64_t)j * k + c]);
  red[threadIdx.x] = m;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + h]);
    __syncthreads();
  }
  const double mall = red[0];
  __syncthreads();
  red[threadIdx.x] = dm;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + h]);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double bound = mall + coef * fabs(sc->eta) * red[0];
    float sv = 1.0f;
    if (bound > 0.0 && isfinite(bound)) {
      int ex;
      frexp(bound, &ex);  // bound = f 2^ex, f in [0.5, 1)
      int p = ex - 14;
      if (p < -60) p = -60;
      sv = ldexpf(1.0f, p);
    }
    scale[c] = sv;
  }
}

// one element of the update: returns the new z; writes V, Z and W in place
__device__ __forceinline__ float nest_elem(float* __restrict__ V, float* __restrict__ Z,
                                           void* __restrict__ W, DT wt, int64_t g, double v,
                                           double z, double st, bool hit, double beta,
                                           double gamma, double alpha, double cz, int z_next,
                                           int accel, float& vout) {
  double vn = v, zn = z, w = z;
  if (accel) {
    vn = beta * v + (1.0 - beta) * z;
    zn = alpha * (z_next ? vn : v) + (1.0 - alpha) * z;
  }
  if (hit) {
    if (accel) vn -= gamma * st;
    zn -= cz * st;
    w -= st;
  }
  vout = (float)vn;
  if (W) {
    if (wt == DT::F64) static_cast<double*>(W)[g] = w;
    else static_cast<float*>(W)[g] = (float)w;
  }
  return (float)zn;
}

template <bool WIDE>
// four waves per SIMD (at most 128 registers; the unconstrained kernel took 134, three waves)
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void nesterov_pack_kernel(
    int64_t n, int k, int64_t ntiles, float* __restrict__ V, float* __restrict__ Z,
    const int64_t* __restrict__ pos, uint32_t stamp, const double* __restrict__ D,
    const IterScalars* __restrict__ sc, double beta, double gamma, double alpha, int z_next,
    int accel, void* __restrict__ W, DT wt, const float* __restrict__ scale, int nq,
    half8* __restrict__ packed, float* __restrict__ part) {
  __shared__ float zt[TILE * 128];
  __shared__ unsigned int mv[128], mz[128];
  const int tid = threadIdx.x;
  for (int c = tid; c < k; c += 256) mv[c] = mz[c] = 0u;
  const double eta = sc->eta;
  const double cz = accel ? (z_next ? alpha * gamma + 1.0 - alpha : 1.0 - alpha) : 1.0;
  const int words = WIDE ? nq * 128 : nq * 64;  // half8 words of one packed tile
  // k a multiple of 8: each thread takes 8 consecutive elements of one row per step (two
  // 16-byte loads of V and of Z) and keeps the maxima of its columns in registers
  const bool vec = (k % 8) == 0;
  float rv[8] = {0, 0, 0, 0, 0, 0, 0, 0}, rz[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  int vcol = -1;  // first of the thread's 8 columns (fixed when 256 * 8 is a multiple of k)
  for (int64_t T = blockIdx.x; T < ntiles; T += gridDim.x) {
    __syncthreads();  // the previous tile's packing has read zt
    if (vec) {
      for (int e0 = tid * 8; e0 < TILE * k; e0 += 256 * 8) {
        const int r = e0 / k, c0 = e0 % k;
        const int64_t i = T * TILE + r;
        float zo[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        if (i < n) {
          const int64_t g = i * k + c0;
          const float4 va = *reinterpret_cast<const float4*>(V + g);
          const float4 vb = *reinterpret_cast<const float4*>(V + g + 4);
          const float4 za = *reinterpret_cast<const float4*>(Z + g);
          const float4 zb = *reinterpret_cast<const float4*>(Z + g + 4);
          const float vv[8] = {va.x, va.y, va.z, va.w, vb.x, vb.y, vb.z, vb.w};
          const float zz[8] = {za.x, za.y, za.z, za.w, zb.x, zb.y, zb.z, zb.w};
          const int64_t p = pos[i];
          const bool hit = (uint32_t)((uint64_t)p >> 32) == stamp;
          const double* Drow = hit ? D + (int64_t)(p & 0xffffffffLL) * k + c0 : nullptr;
          float vo[8];
#pragma unroll
          for (int j = 0; j < 8; ++j) {
            const double st = hit ? eta * Drow[j] : 0.0;
            zo[j] = nest_elem(V, Z, W, wt, g + j, (double)vv[j], (double)zz[j], st, hit, beta,
                              gamma, alpha, cz, z_next, accel, vo[j]);
          }
          if (accel) {
            *reinterpret_cast<float4*>(V + g) = make_float4(vo[0], vo[1], vo[2], vo[3]);
            *reinterpret_cast<float4*>(V + g + 4) = make_float4(vo[4], vo[5], vo[6], vo[7]);
          }
          *reinterpret_cast<float4*>(Z + g) = make_float4(zo[0], zo[1], zo[2], zo[3]);
          *reinterpret_cast<float4*>(Z + g + 4) = make_float4(zo[4], zo[5], zo[6], zo[7]);
          if ((256 * 8) % k == 0) {
            vcol = c0;
#pragma unroll
            for (int j = 0; j < 8; ++j) {
              rv[j] = fmaxf(rv[j], fabsf(accel ? vo[j] : zo[j]));
              rz[j] = fmaxf(rz[j], fabsf(zo[j]));
            }
          } else {
#pragma unroll
            for (int j = 0; j < 8; ++j) {
              atomicMax(&mv[c0 + j], __float_as_uint(fabsf(accel ? vo[j] : zo[j])));
              atomicMax(&mz[c0 + j], __float_as_uint(fabsf(zo[j])));
            }
          }
        }
#pragma unroll
        for (int j = 0; j < 8; ++j) zt[r * k + c0 + j] = zo[j];
      }
    } else {
    for (int e = tid; e < TILE * k; e += 256) {
      const int64_t i = T * TILE + e / k;
      const int c = e % k;
      float zo = 0.0f;
      if (i < n) {
        const int64_t g = i * k + c;
        const double v = (double)V[g], z = (double)Z[g];
        double vn = v, zn = z, w = z;
        if (accel) {
          vn = beta * v + (1.0 - beta) * z;
          zn = alpha * (z_next ? vn : v) + (1.0 - alpha) * z;
        }
        const int64_t p = pos[i];
        if ((uint32_t)((uint64_t)p >> 32) == stamp) {
          const double st = eta * D[(int64_t)(p & 0xffffffffLL) * k + c];
          if (accel) vn -= gamma * st;
          zn -= cz * st;
          w -= st;
        }
        if (accel) {
          V[g] = (float)vn;
          atomicMax(&mv[c], __float_as_uint(fabsf((float)vn)));
        }
        Z[g] = (float)zn;
        zo = (float)zn;
        atomicMax(&mz[c], __float_as_uint(fabsf(zo)));
        if (W) {
          if (wt == DT::F64) static_cast<double*>(W)[g] = w;
          else static_cast<float*>(W)[g] = (float)w;
        }
      }
      zt[(e / k) * k + c] = zo;
    }
    }
    __syncthreads();
    for (int e = tid; e < words; e += 256) {
      const int lane = e % 64;
      half8 h;
      if constexpr (WIDE) {
        const int t = (e / 64) % 2, q = e / 128;
        const int rhs = q * 32 + lane % 32;
        const float inv = rhs < k ? 1.0f / scale[rhs] : 0.0f;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          const int col = wide_col(t, 8 * (lane / 32) + j);
          const float x = rhs < k ? zt[col * k + rhs] : 0.0f;
          h[j] = (_Float16)(rhs < k ? (float)((double)x * (double)inv) : 0.0f);
        }
        packed[((T * nq + q) * 2 + t) * 64 + lane] = h;
      } else {
        const int q = e / 64;
        const int rhs = q * 16 + lane % 16;
        const float inv = rhs < k ? 1.0f / scale[rhs] : 0.0f;
#pragma unroll
        for (int m = 0; m < 8; ++m) {
          const int col = slot_col(lane, m);
          const float x = rhs < k ? zt[col * k + rhs] : 0.0f;
          h[m] = (_Float16)(rhs < k ? (float)((double)x * (double)inv) : 0.0f);
        }
        packed[(T * nq + q) * 64 + lane] = h;
      }
    }
  }
  if (vcol >= 0) {
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      atomicMax(&mv[vcol + j], __float_as_uint(rv[j]));
      atomicMax(&mz[vcol + j], __float_as_uint(rz[j]));
    }
  }
  __syncthreads();
  for (int c = tid; c < k; c += 256) {
    part[((int64_t)blockIdx.x * 2 + 0) * k + c] = __uint_as_float(accel ? mv[c] : mz[c]);
    part[((int64_t)blockIdx.x * 2 + 1) * k + c] = __uint_as_float(mz[c]);
  }
}

}  // namespace

// ---------------------------------------------------------------- batches
// step-I partial sums of the work-queue items back to G[p][i][c] (+ epilogue)
__global__ void mkq_reduce_kernel(const float* __restrict__ part, const int64_t* __restrict__ item_start,
                                  const int* __restrict__ nchunk, int64_t b, int k, int rows_per_wg,
                                  KbEpilogue ep, double* __restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= b * k) return;
  const int pb = blockIdx.y;
  const int64_t i = e / k;
  const int c = (int)(e % k);
  const int rw = (int)(i / rows_per_wg);
  const int nc = nchunk[pb];
  const int64_t first = item_start[pb] + (int64_t)rw * nc;
  double s = 0.0;
  for (int j = 0; j < nc; ++j) s += (double)part[((first + j) * rows_per_wg + (i - (int64_t)rw * rows_per_wg)) * k + c];
  auto ld = [](const void* p, DT t, int64_t j) {
    return t == DT::F64 ? static_cast<const double*>(p)[j] : (double)static_cast<const float*>(p)[j];
  };
  const int64_t* i1 = ep.e1idx ? ep.e1idx + (int64_t)pb * ep.bsIdx : nullptr;
  const int64_t* i2 = ep.e2idx ? ep.e2idx + (int64_t)pb * ep.bsIdx : nullptr;
  if (ep.E1) s += ep.a1 * ld(ep.E1, ep.e1t, (i1 ? i1[i] : i) * ep.lde1 + c);
  if (ep.E2) s += ep.a2 * ld(ep.E2, ep.e2t, (i2 ? i2[i] : i) * ep.lde2 + c);
  out[(int64_t)pb * b * k + e] = s;
}

// the XCD range counters of a work queue (a kernel, not a memset, so that a captured graph
// holds no memset node)
__global__ void zero_queue_counters_kernel(int* p) {
  if (threadIdx.x < QXCDS) p[threadIdx.x * QCOUNTER_STRIDE] = 0;
}

// ---------------------------------------------------------------- public launchers
size_t mfma_pack_bytes(int64_t n, int d, int k) {
  const int64_t nt = (n + TILE - 1) / TILE;
  const int KS = ksteps(d);
  return (size_t)nt * TILE * ROWVEC * 2 + (size_t)nt * 2 * KS * 64 * 16 +
         (size_t)nt * ((k + 15) / 16) * 64 * 16;
}

adasap_status_t mfma_pack_create(MfmaPack& pk, int64_t n, int d, int k, const void* X, DT xt,
                                 int kern, double ell, hipStream_t s) {
  if (d < 1 || d > 16) {
    set_error("matrix-core kernel-block products need 1 <= d <= 16");
    return ADASAP_ERR_INVALID_ARG;
  }
  (void)k;
  pk.n = n;
  pk.d = d;
  pk.kern = kern;
  pk.ell = ell;
  pk.ntiles = (n + TILE - 1) / TILE;
  pk.sigma = sigma_for(kern, ell);
  const int64_t npad = pk.ntiles * TILE;
  const int KS = ksteps(d);
  ADASAP_TRY(pk.centre.ensure((size_t)d * sizeof(double)));
  ADASAP_TRY(pk.rowv.ensure((size_t)npad * ROWVEC * 2));
  ADASAP_TRY(pk.cols.ensure((size_t)pk.ntiles * 2 * KS * 64 * 16));
  ADASAP_TRY(pk.flag.ensure(sizeof(int)));
  const int nblk = (int)((n + 4095) / 4096);
  ADASAP_TRY(pk.tmp.ensure((size_t)(nblk > 0 ? nblk : 1) * d * sizeof(double)));
  hipLaunchKernelGGL(mean_partial_kernel, dim3(nblk), dim3(256), 0, s, X, xt, n, d, pk.tmp.as<double>());
  ADASAP_LAUNCH_CHECK();
  hipLaunchKernelGGL(mean_final_kernel, dim3(1), dim3(64), 0, s, pk.tmp.as<double>(), nblk, d, n,
                     pk.centre.as<double>());
  ADASAP_LAUNCH_CHECK();
  ADASAP_HIP(hipMemsetAsync(pk.flag.p, 0, sizeof(int), s));
  hipLaunchKernelGGL(rowpack_kernel, dim3((unsigned)((npad + 255) / 256)), dim3(256), 0, s, X, xt,
                     n, npad, d, pk.centre.as<double>(), pk.sigma, pk.rowv.as<_Float16>(),
                     pk.flag.as<int>());
  ADASAP_LAUNCH_CHECK();
  const int64_t nfr = pk.ntiles * 2 * KS * 64;
  hipLaunchKernelGGL(colpack_kernel, dim3((unsigned)((nfr + 255) / 256)), dim3(256), 0, s,
                     pk.rowv.as<_Float16>(), nullptr, n, pk.ntiles, d, KS, pk.cols.as<half8>(),
                     nullptr);
  ADASAP_LAUNCH_CHECK();
  int flag = 0;
  ADASAP_HIP(hipMemcpyAsync(&flag, pk.flag.p, sizeof(int), hipMemcpyDeviceToHost, s));
  ADASAP_HIP(hipStreamSynchronize(s));
  if (flag) {
    set_error("scaled coordinates exceed the float16 range of the matrix-core path "
              "(lengthscale too small for the data spread); use FP32 or FP64 precision");
    return ADASAP_ERR_UNSUPPORTED;
  }
  return ADASAP_OK;
}

adasap_status_t mfma_pack_block(const MfmaPack& pk, const int64_t* B, int64_t b, DevBuf& colsB,
                                hipStream_t s) {
  const int KS = ksteps(pk.d);
  const int64_t nt = (b + TILE - 1) / TILE;
  ADASAP_TRY(colsB.ensure((size_t)nt * 2 * KS * 64 * 16));
  const int64_t nfr = nt * 2 * KS * 64;
  hipLaunchKernelGGL(colpack_kernel, dim3((unsigned)((nfr + 255) / 256)), dim3(256), 0, s,
                     pk.rowv.as<_Float16>(), B, b, nt, pk.d, KS, colsB.as<half8>(), nullptr);
  ADASAP_LAUNCH_CHECK();
  return ADASAP_OK;
}

adasap_status_t mfma_product(const MfmaPack& pk, const int64_t* ridx, int64_t m,
                             const void* colsB, int64_t ncols, const void* R, DT rt, int k,
                             int mode, void* out, DT ot, const KbEpilogue& ep, MfmaWork& w,
                             hipStream_t s) {
  const bool all_cols = colsB == nullptr;
  const int64_t nt = all_cols ? pk.ntiles : (ncols + TILE - 1) / TILE;
  const int64_t rows = all_cols ? pk.n : ncols;
  // the float16 mode with 17 to 64 right-hand sides runs on 32x32x16 MFMAs (more would not
  // fit two waves per SIMD without scratch)
  if (mode == MODE_F16 && k > 16 && k <= 64) mode = MODE_F16W;
  RhsDesc rd;
  ADASAP_TRY(pack_rhs(R, rt, rows, k, k, nullptr, nt, mode, w.rhs, w.scale, w.tmp, rd, s));
  if (w.wait_ev) ADASAP_HIP(hipStreamWaitEvent(s, w.wait_ev, 0));
  return mk_run(all_cols ? pk.cols.as<half8>() : static_cast<const half8*>(colsB), nt,
                pk.rowv.as<half8>(), ridx, m, pk.d, pk.kern, rd, k, out, ot, ep, w.part, s, w.ev0,
                w.ev1, 0, w.cap_cus);
}

adasap_status_t mfma_product_packed(const MfmaPack& pk, const int64_t* ridx, int64_t m,
                                    const RhsPacked& rp, int k, void* out, DT ot,
                                    const KbEpilogue& ep, MfmaWork& w, hipStream_t s) {
  RhsDesc rd{rp.mode, rp.nq, rp.p, rp.scale};
  if (w.wait_ev) ADASAP_HIP(hipStreamWaitEvent(s, w.wait_ev, 0));
  return mk_run(pk.cols.as<half8>(), pk.ntiles, pk.rowv.as<half8>(), ridx, m, pk.d, pk.kern, rd,
                k, out, ot, ep, w.part, s, w.ev0, w.ev1, 0, w.cap_cus);
}

adasap_status_t mfma_pack_rhs_full(const MfmaPack& pk, const void* R, DT rt, int k, int mode,
                                   MfmaWork& w, RhsPacked& rp, hipStream_t s) {
  RhsDesc rd;
  ADASAP_TRY(pack_rhs(R, rt, pk.n, k, k, nullptr, pk.ntiles, mode, w.rhs, w.scale, w.tmp, rd, s));
  rp.mode = rd.mode;
  rp.nq = rd.nq;
  rp.p = rd.p;
  rp.scale = rd.scale;
  return ADASAP_OK;
}

adasap_status_t mfma_points(const MfmaPack& pk, const void* Xq, DT xt, int64_t m, DevBuf& rowq,
                            hipStream_t s) {
  const int64_t mpad = (m + 15) / 16 * 16;
  ADASAP_TRY(rowq.ensure((size_t)mpad * ROWVEC * 2));
  ADASAP_TRY(const_cast<MfmaPack&>(pk).flag.ensure(sizeof(int)));
  ADASAP_HIP(hipMemsetAsync(pk.flag.p, 0, sizeof(int), s));
  hipLaunchKernelGGL(rowpack_kernel, dim3((unsigned)((mpad + 255) / 256)), dim3(256), 0, s, Xq, xt,
                     m, mpad, pk.d, pk.centre.as<double>(), pk.sigma, rowq.as<_Float16>(),
                     pk.flag.as<int>());
  ADASAP_LAUNCH_CHECK();
  int flag = 0;
  ADASAP_HIP(hipMemcpyAsync(&flag, pk.flag.p, sizeof(int), hipMemcpyDeviceToHost, s));
  ADASAP_HIP(hipStreamSynchronize(s));
  if (flag) {
    set_error("query points exceed the float16 range of the matrix-core path");
    return ADASAP_ERR_UNSUPPORTED;
  }
  return ADASAP_OK;
}

adasap_status_t mfma_product_rows(const MfmaPack& pk, const void* rowq, int64_t m, const void* R,
                                  DT rt, int k, int mode, void* out, DT ot, MfmaWork& w,
                                  hipStream_t s, double kscale) {
  RhsDesc rd;
  ADASAP_TRY(pack_rhs(R, rt, pk.n, k, k, nullptr, pk.ntiles, mode, w.rhs, w.scale, w.tmp, rd, s));
  KbEpilogue ep;
  ep.kscale = kscale;
  return mk_run(pk.cols.as<half8>(), pk.ntiles, static_cast<const half8*>(rowq), nullptr, m, pk.d,
                pk.kern, rd, k, out, ot, ep, w.part, s);
}

adasap_status_t mfma_batch_pack_create(MfmaBatchPack& bp, int P, const int64_t* n, const int* d,
                                       const void* const* X, DT xt, const double* ell, int kern,
                                       hipStream_t s) {
  bp.P = P;
  bp.kern = kern;
  bp.n.assign(n, n + P);
  bp.d.assign(d, d + P);
  bp.ntiles.resize(P);
  bp.row_off.resize(P);
  bp.col_off.resize(P);
  int64_t rows = 0, cols = 0;
  for (int p = 0; p < P; ++p) {
    if (d[p] < 1 || d[p] > 16) {
      set_error("batched solves need 1 <= d <= 16 for every problem");
      return ADASAP_ERR_INVALID_ARG;
    }
    bp.ntiles[p] = (n[p] + TILE - 1) / TILE;
    bp.row_off[p] = rows;
    bp.col_off[p] = cols;
    rows += bp.ntiles[p] * TILE;
    cols += bp.ntiles[p] * 2 * 2 * 64;  // two K-steps for every batched problem
  }
  bp.rows_total = rows;
  ADASAP_TRY(bp.rowv.ensure((size_t)rows * ROWVEC * 2));
  ADASAP_TRY(bp.cols.ensure((size_t)cols * 16));
  ADASAP_TRY(bp.flag.ensure(sizeof(int)));
  ADASAP_TRY(bp.centre.ensure((size_t)16 * sizeof(double)));
  ADASAP_TRY(bp.dvec.ensure((size_t)P * sizeof(int)));
  ADASAP_TRY(bp.col_off_dev.ensure((size_t)P * sizeof(int64_t)));
  ADASAP_TRY(bp.rhs_off_dev.ensure((size_t)P * sizeof(int64_t)));
  ADASAP_HIP(hipMemcpyAsync(bp.dvec.p, d, (size_t)P * sizeof(int), hipMemcpyHostToDevice, s));
  ADASAP_HIP(hipMemcpyAsync(bp.col_off_dev.p, bp.col_off.data(), (size_t)P * sizeof(int64_t),
                            hipMemcpyHostToDevice, s));
  std::vector<int64_t> rhs_off(P);
  for (int p = 0; p < P; ++p) rhs_off[p] = bp.row_off[p] * (int64_t)sizeof(float);  // k = 1 float32
  ADASAP_HIP(hipMemcpyAsync(bp.rhs_off_dev.p, rhs_off.data(), (size_t)P * sizeof(int64_t),
                            hipMemcpyHostToDevice, s));
  ADASAP_HIP(hipMemsetAsync(bp.flag.p, 0, sizeof(int), s));
  DevBuf tmp;
  for (int p = 0; p < P; ++p) {
    const int nblk = (int)((n[p] + 4095) / 4096);
    ADASAP_TRY(tmp.ensure((size_t)nblk * d[p] * sizeof(double)));
    hipLaunchKernelGGL(mean_partial_kernel, dim3(nblk), dim3(256), 0, s, X[p], xt, n[p], d[p],
                       tmp.as<double>());
    hipLaunchKernelGGL(mean_final_kernel, dim3(1), dim3(64), 0, s, tmp.as<double>(), nblk, d[p],
                       n[p], bp.centre.as<double>());
    const int64_t npad = bp.ntiles[p] * TILE;
    _Float16* rv = bp.rowv.as<_Float16>() + bp.row_off[p] * ROWVEC;
    hipLaunchKernelGGL(rowpack_kernel, dim3((unsigned)((npad + 255) / 256)), dim3(256), 0, s, X[p],
                       xt, n[p], npad, d[p], bp.centre.as<double>(), sigma_for(kern, ell[p]), rv,
                       bp.flag.as<int>());
    const int64_t nfr = bp.ntiles[p] * 2 * 2 * 64;
    hipLaunchKernelGGL(colpack_kernel, dim3((unsigned)((nfr + 255) / 256)), dim3(256), 0, s, rv,
                       nullptr, n[p], bp.ntiles[p], d[p], 2, bp.cols.as<half8>() + bp.col_off[p],
                       nullptr);
    ADASAP_LAUNCH_CHECK();
    ADASAP_HIP(hipStreamSynchronize(s));  // the centre buffer is reused by the next problem
  }
  int flag = 0;
  ADASAP_HIP(hipMemcpy(&flag, bp.flag.p, sizeof(int), hipMemcpyDeviceToHost));
  if (flag) {
    set_error("scaled coordinates exceed the float16 range of the matrix-core path");
    return ADASAP_ERR_UNSUPPORTED;
  }
  return ADASAP_OK;
}

adasap_status_t mfma_batch_pack_blocks(const MfmaBatchPack& bp, const int64_t* B, int64_t b,
                                       DevBuf& colsB, hipStream_t s) {
  const int64_t nt = (b + TILE - 1) / TILE;
  const int64_t nfr = nt * 2 * 2 * 64;
  ADASAP_TRY(colsB.ensure((size_t)bp.P * nfr * 16));
  hipLaunchKernelGGL(colpack_kernel, dim3((unsigned)((nfr + 255) / 256), bp.P), dim3(256), 0, s,
                     bp.rowv.as<_Float16>(), B, b, nt, 0, 2, colsB.as<half8>(), bp.dvec.as<int>());
  ADASAP_LAUNCH_CHECK();
  return ADASAP_OK;
}

adasap_status_t mfma_batch_block_product(const MfmaBatchPack& bp, const int64_t* B, int64_t b,
                                         const void* colsB, const double* R, int k, int mode,
                                         double* out, const KbEpilogue& ep, MfmaWork& w,
                                         hipStream_t s) {
  const int P = bp.P;
  const int64_t nt = (b + TILE - 1) / TILE;
  RhsDesc rd;
  rd.mode = mode;
  if (mode == MODE_F32V) {
    const int kc = k == 1 ? 1 : (k == 2 ? 2 : 4);
    const int64_t npad = nt * TILE;
    ADASAP_TRY(w.rhs.ensure((size_t)P * npad * kc * sizeof(float)));
    const int64_t tot = npad * kc;
    const dim3 g((unsigned)((tot + 255) / 256), P);
    if (kc == 1) hipLaunchKernelGGL(rhspack32_kernel<1>, g, dim3(256), 0, s, R, DT::F64, b, k, k, nullptr, npad, w.rhs.as<float>());
    else if (kc == 2) hipLaunchKernelGGL(rhspack32_kernel<2>, g, dim3(256), 0, s, R, DT::F64, b, k, k, nullptr, npad, w.rhs.as<float>());
    else hipLaunchKernelGGL(rhspack32_kernel<4>, g, dim3(256), 0, s, R, DT::F64, b, k, k, nullptr, npad, w.rhs.as<float>());
    ADASAP_LAUNCH_CHECK();
    rd.nq = kc;
    rd.p = w.rhs.p;
    rd.scale = nullptr;
  } else {
    const int nq = (k + 15) / 16;
    const int parts = mode == MODE_F16X3 ? 2 : 1;
    ADASAP_TRY(w.rhs.ensure((size_t)P * nt * nq * parts * 64 * 16));
    ADASAP_TRY(w.scale.ensure((size_t)P * k * sizeof(float)));
    const int64_t rpb = colmax_rows_per_block(b);
    const int nblk = (int)((b + rpb - 1) / rpb);
    ADASAP_TRY(w.tmp.ensure((size_t)P * nblk * k * sizeof(float)));
    hipLaunchKernelGGL(colmax_partial_kernel, dim3(nblk, P), dim3(256), 0, s, R, DT::F64, b, k, k,
                       w.tmp.as<float>(), rpb);
    hipLaunchKernelGGL(colmax_final_kernel, dim3(k, P), dim3(256), 0, s, w.tmp.as<float>(), nblk, k,
                       w.scale.as<float>());
    const int64_t tot = nt * nq * 64;
    hipLaunchKernelGGL(rhspack16_kernel, dim3((unsigned)((tot + 255) / 256), P), dim3(256), 0, s, R,
                       DT::F64, b, k, k, nullptr, w.scale.as<float>(), nt, nq, parts,
                       w.rhs.as<half8>());
    ADASAP_LAUNCH_CHECK();
    rd.nq = nq;
    rd.p = w.rhs.p;
    rd.scale = w.scale.as<float>();
  }
  const int RT = rt_of(rd.mode, rd.nq);
  const int rows_per_wg = WAVES * RT * 16;
  const int rwg = (int)((b + rows_per_wg - 1) / rows_per_wg);
  // about 1024 workgroups over the batch: one column split per problem at 256 problems, so
  // the reduction reads one partial per entry
  int splits = (int)((1024 / P + rwg - 1) / rwg);
  if (splits > nt) splits = (int)nt;
  if (splits < 1) splits = 1;
  int64_t tps = (nt + splits - 1) / splits;
  splits = (int)((nt + tps - 1) / tps);
  ADASAP_TRY(w.part.ensure((size_t)P * splits * b * k * sizeof(float)));
  MkArgs a{};
  a.colA = static_cast<const half8*>(colsB);
  a.rowv = bp.rowv.as<half8>();
  a.ridx = B;
  a.m = b;
  a.rhs = rd.p;
  a.ntiles = nt;
  a.tiles_per_split = tps;
  a.splits = splits;
  a.rwg = rwg;
  a.xcd_map = 0;
  a.part = w.part.as<float>();
  a.k = k;
  a.p = matern_factor(bp.kern);
  a.bs_colA = nt * 2 * 2 * 64;
  a.bs_ridx = b;
  if (mode == MODE_F32V) a.bs_rhs = nt * TILE * rd.nq * (int64_t)sizeof(float);
  else a.bs_rhs = nt * rd.nq * (mode == MODE_F16X3 ? 2 : 1) * 64 * 16;
  a.bs_part = (int64_t)splits * b * k;
  const dim3 grid(rwg * splits, P);
  if (mode == MODE_F32V) {
    // every problem has two K-steps (d <= 16): all four 16-slot K-slices
    ADASAP_TRY(disp_vwide(a, 2, 4, bp.kern, rd.nq, grid, s));
  } else switch (bp.kern) {
    case ADASAP_RBF: disp_mode_grid<2, ADASAP_RBF>(a, rd.mode, rd.nq, grid, s); break;
    case ADASAP_MATERN12: disp_mode_grid<2, ADASAP_MATERN12>(a, rd.mode, rd.nq, grid, s); break;
    case ADASAP_MATERN32: disp_mode_grid<2, ADASAP_MATERN32>(a, rd.mode, rd.nq, grid, s); break;
    default: disp_mode_grid<2, ADASAP_MATERN52>(a, rd.mode, rd.nq, grid, s); break;
  }
  ADASAP_LAUNCH_CHECK();
  hipLaunchKernelGGL(mk_reduce_kernel, dim3((unsigned)((b * k + 255) / 256), P), dim3(256), 0, s,
                     w.part.as<float>(), splits, b, k, rd.scale, ep, out, DT::F64);
  ADASAP_LAUNCH_CHECK();
  return ADASAP_OK;
}

template <int RT>
static adasap_status_t mkq_launch(int kern, int grid, const MkArgs& a, hipStream_t s) {
  switch (kern) {
    case ADASAP_RBF: hipLaunchKernelGGL((mkq_kernel<2, ADASAP_RBF, MODE_F32V, 1, RT>), dim3(grid), dim3(256), 0, s, a); break;
    case ADASAP_MATERN12: hipLaunchKernelGGL((mkq_kernel<2, ADASAP_MATERN12, MODE_F32V, 1, RT>), dim3(grid), dim3(256), 0, s, a); break;
    case ADASAP_MATERN32: hipLaunchKernelGGL((mkq_kernel<2, ADASAP_MATERN32, MODE_F32V, 1, RT>), dim3(grid), dim3(256), 0, s, a); break;
    default: hipLaunchKernelGGL((mkq_kernel<2, ADASAP_MATERN52, MODE_F32V, 1, RT>), dim3(grid), dim3(256), 0, s, a); break;
  }
  ADASAP_LAUNCH_CHECK();
  return ADASAP_OK;
}

adasap_status_t mfma_batch_queue_create(const MfmaBatchPack& bp, int64_t b, int64_t chunk_tiles,
                                        int rt, MfmaQueue& q, hipStream_t s) {
  if (rt != 2 && rt != 4) {
    set_error("batched step I: row tiles per wave must be 2 or 4");
    return ADASAP_ERR_INVALID_ARG;
  }
  const int P = bp.P;
  const int rows_per_wg = WAVES * rt * 16;
  const int rwg = (int)((b + rows_per_wg - 1) / rows_per_wg);
  // Partial-sum slots keep the problem-major, row-workgroup-major order that the reduction
  // reads (start[p] + rw * nc + c).  The queue itself runs tile range by tile range, the row
  // workgroups of a range adjacent, cut into QXCDS contiguous ranges of about equal tile counts.
  std::vector<MkItem> items;
  std::vector<int64_t> start(P);
  std::vector<int> nch(P);
  int64_t total_tiles = 0, nslots = 0;
  for (int p = 0; p < P; ++p) {
    const int64_t nt = bp.ntiles[p];
    const int nc = (int)((nt + chunk_tiles - 1) / chunk_tiles);
    start[p] = nslots;
    nch[p] = nc;
    nslots += (int64_t)rwg * nc;
    total_tiles += nt;
  }
  if (nslots > INT32_MAX) {
    set_error("batched step I: work queue too long");
    return ADASAP_ERR_INVALID_ARG;
  }
  int qcount[QXCDS] = {0};
  int64_t done_tiles = 0;
  for (int p = 0; p < P; ++p) {
    const int64_t nt = bp.ntiles[p];
    for (int c = 0; c < nch[p]; ++c) {
      MkItem it{};
      it.prob = p;
      it.T0 = (int64_t)c * chunk_tiles;
      it.T1 = it.T0 + chunk_tiles < nt ? it.T0 + chunk_tiles : nt;
      int x = total_tiles > 0 ? (int)(done_tiles * QXCDS / total_tiles) : 0;
      if (x >= QXCDS) x = QXCDS - 1;
      done_tiles += it.T1 - it.T0;
      for (int rw = 0; rw < rwg; ++rw) {
        it.rw = rw;
        it.slot = (int)(start[p] + (int64_t)rw * nch[p] + c);
        items.push_back(it);
        ++qcount[x];
      }
    }
  }
  q.qbeg[0] = 0;
  for (int x = 0; x < QXCDS; ++x) q.qbeg[x + 1] = q.qbeg[x] + qcount[x];
  q.nitems = (int)items.size();
  q.rows_per_wg = rows_per_wg;
  q.rt = rt;
  ADASAP_TRY(q.items.ensure(items.size() * sizeof(MkItem)));
  ADASAP_TRY(q.item_start.ensure((size_t)P * sizeof(int64_t)));
  ADASAP_TRY(q.nchunk.ensure((size_t)P * sizeof(int)));
  ADASAP_TRY(q.counter.ensure((size_t)QXCDS * QCOUNTER_STRIDE * sizeof(int)));
  ADASAP_HIP(hipMemcpyAsync(q.items.p, items.data(), items.size() * sizeof(MkItem),
                            hipMemcpyHostToDevice, s));
  ADASAP_HIP(hipMemcpyAsync(q.item_start.p, start.data(), (size_t)P * sizeof(int64_t),
                            hipMemcpyHostToDevice, s));
  ADASAP_HIP(hipMemcpyAsync(q.nchunk.p, nch.data(), (size_t)P * sizeof(int), hipMemcpyHostToDevice, s));
  ADASAP_HIP(hipStreamSynchronize(s));
  return ADASAP_OK;
}

adasap_status_t mfma_batch_stepI(const MfmaBatchPack& bp, MfmaQueue& q, const int64_t* B, int64_t b,
                                 const float* Z, double* out, const KbEpilogue& ep, MfmaWork& w,
                                 hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
  ADASAP_TRY(w.part.ensure((size_t)q.nitems * q.rows_per_wg * sizeof(float)));
  MkArgs a{};
  a.colA = bp.cols.as<half8>();
  a.rowv = bp.rowv.as<half8>();
  a.ridx = B;
  a.m = b;
  a.rhs = Z;
  a.k = 1;
  a.p = matern_factor(bp.kern);
  a.part = w.part.as<float>();
  a.bs_ridx = b;
  a.items = q.items.as<MkItem>();
  a.nitems = q.nitems;
  a.counter = q.counter.as<int>();
  a.colA_off = bp.col_off_dev.as<int64_t>();
  a.rhs_off = bp.rhs_off_dev.as<int64_t>();
  for (int x = 0; x <= QXCDS; ++x) a.qbeg[x] = q.qbeg[x];
  hipLaunchKernelGGL(zero_queue_counters_kernel, dim3(1), dim3(64), 0, s, a.counter);
  ADASAP_LAUNCH_CHECK();
  int dev = 0, cus = 256;
  ADASAP_HIP(hipGetDevice(&dev));
  ADASAP_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  // persistent workgroups (two or four per CU, within the launch bounds of four), each
  // draining its XCD's range of the queue; every range needs at least one workgroup
  const int grid = cus * (q.wg_per_cu == 4 ? 4 : 2);
  if (grid < QXCDS) {
    set_error("batched step I: fewer persistent workgroups than queue ranges");
    return ADASAP_ERR_INVALID_ARG;
  }
  if (ev0) ADASAP_HIP(hipEventRecord(ev0, s));
  if (q.rt == 2) ADASAP_TRY(mkq_launch<2>(bp.kern, grid, a, s));
  else ADASAP_TRY(mkq_launch<4>(bp.kern, grid, a, s));
  if (ev1) ADASAP_HIP(hipEventRecord(ev1, s));
  hipLaunchKernelGGL(mkq_reduce_kernel, dim3((unsigned)((b + 255) / 256), bp.P), dim3(256), 0, s,
                     w.part.as<float>(), q.item_start.as<int64_t>(), q.nchunk.as<int>(), b, 1,
                     q.rows_per_wg, ep, out);
  ADASAP_LAUNCH_CHECK();
  return ADASAP_OK;
}

adasap_status_t mfma_batch_residual(const MfmaBatchPack& bp, int p, const void* W, DT wt,
                                    const void* Y, DT yt, double lam, double* res, MfmaWork& w,
                                    hipStream_t s) {
  RhsDesc rd;
  ADASAP_TRY(pack_rhs(W, wt, bp.n[p], 1, 1, nullptr, bp.ntiles[p], MODE_F16X3, w.rhs, w.scale,
                      w.tmp, rd, s));
  KbEpilogue ep;
  ep.E1 = W;
  ep.e1t = wt;
  ep.lde1 = 1;
  ep.a1 = lam;
  ep.E2 = Y;
  ep.e2t = yt;
  ep.lde2 = 1;
  ep.a2 = -1.0;
  return mk_run(bp.cols.as<half8>() + bp.col_off[p], bp.ntiles[p],
                bp.rowv.as<half8>() + bp.row_off[p] * 8, nullptr, bp.n[p], bp.d[p], bp.kern, rd, 1,
                res, DT::F64, ep, w.part, s, nullptr, nullptr, 2);
}


// ---------------------------------------------------------------- fused update launchers
namespace {
int fused_nwg(int64_t ntiles) { return (int)(ntiles < FU_TILES_MAX ? (ntiles > 0 ? ntiles : 1) : FU_TILES_MAX); }
}  // namespace

adasap_status_t fused_init(const MfmaPack& pk, FusedUpd& f, int k, const float* V, const float* Z,
                           MfmaWork& w, hipStream_t s) {
  if (k < 1 || k > 128) {
    set_error("the fused update packs 1 to 128 right-hand sides");
    return ADASAP_ERR_INVALID_ARG;
  }
  const int mode = (k > 16 && k <= 64) ? MODE_F16W : MODE_F16;
  f.nwg = fused_nwg(pk.ntiles);
  ADASAP_TRY(f.part.ensure((size_t)f.nwg * 2 * k * sizeof(float)));
  if (!f.pos.p || f.pos.bytes < (size_t)pk.n * sizeof(int64_t)) {
    ADASAP_TRY(f.pos.ensure((size_t)pk.n * sizeof(int64_t)));
    ADASAP_HIP(hipMemsetAsync(f.pos.p, 0xff, (size_t)pk.n * sizeof(int64_t), s));
  }
  RhsDesc rd;
  ADASAP_TRY(pack_rhs(Z, DT::F32, pk.n, k, k, nullptr, pk.ntiles, mode, f.packed, f.scale, w.tmp, rd, s));
  f.mode = rd.mode;
  f.nq = rd.nq;
  hipLaunchKernelGGL(vzmax_partial_kernel, dim3(f.nwg), dim3(256), 0, s, pk.n, k, pk.ntiles, V, Z,
                     f.part.as<float>());
  ADASAP_LAUNCH_CHECK();
  return ADASAP_OK;
}

RhsPacked fused_rhs(const FusedUpd& f) {
  RhsPacked rp;
  rp.mode = f.mode;
  rp.nq = f.nq;
  rp.p = f.packed.p;
  rp.scale = f.scale.as<float>();
  return rp;
}

adasap_status_t fused_update(const MfmaPack& pk, FusedUpd& f, int k, const int64_t* B, int64_t b,
                             const double* D, const IterScalars* sc, const NestCoef& c, float* V,
                             float* Z, void* W, DT wt, hipStream_t s) {
  ++f.stamp;
  if (f.stamp == 0xffffffffu) f.stamp = 1;  // all ones marks rows never sampled
  hipLaunchKernelGGL(pos_scatter_kernel, dim3((unsigned)((b + 255) / 256)), dim3(256), 0, s, b, B,
                     f.stamp, f.pos.as<int64_t>());
  ADASAP_LAUNCH_CHECK();
  const double cz = c.accel ? (c.z_uses_v_next ? c.alpha * c.gamma + 1.0 - c.alpha : 1.0 - c.alpha) : 1.0;
  const double coef = c.accel ? (c.gamma > cz ? c.gamma : cz) : 1.0;
  // column maxima of |D| in coalesced row blocks, then the scales
  const int64_t rpb = colmax_rows_per_block(b);
  const int dblk = (int)((b + rpb - 1) / rpb);
  ADASAP_TRY(f.dpart.ensure((size_t)(dblk > 0 ? dblk : 1) * k * sizeof(float)));
  if (dblk > 0) {
    hipLaunchKernelGGL(colmax_partial_kernel, dim3(dblk), dim3(256), 0, s, D, DT::F64, b, k,
                       (int64_t)k, f.dpart.as<float>(), rpb);
    ADASAP_LAUNCH_CHECK();
  }
  hipLaunchKernelGGL(fused_scale_kernel, dim3(k), dim3(256), 0, s, f.nwg, k, f.part.as<float>(), dblk,
                     f.dpart.as<float>(), sc, coef, f.scale.as<float>());
  ADASAP_LAUNCH_CHECK();
  if (f.mode == MODE_F16W)
    hipLaunchKernelGGL(nesterov_pack_kernel<true>, dim3(f.nwg), dim3(256), 0, s, pk.n, k, pk.ntiles, V,
                       Z, f.pos.as<int64_t>(), f.stamp, D, sc, c.beta, c.gamma, c.alpha,
                       c.z_uses_v_next, c.accel, W, wt, f.scale.as<float>(), f.nq,
                       f.packed.as<half8>(), f.part.as<float>());
  else
    hipLaunchKernelGGL(nesterov_pack_kernel<false>, dim3(f.nwg), dim3(256), 0, s, pk.n, k, pk.ntiles,
                       V, Z, f.pos.as<int64_t>(), f.stamp, D, sc, c.beta, c.gamma, c.alpha,
                       c.z_uses_v_next, c.accel, W, wt, f.scale.as<float>(), f.nq,
                       f.packed.as<half8>(), f.part.as<float>());
  ADASAP_LAUNCH_CHECK();
  return ADASAP_OK;
}

int mfma_mode_f16() { return MODE_F16; }
int mfma_mode_f16x3() { return MODE_F16X3; }
int mfma_mode_f32v() { return MODE_F32V; }

}  // namespace adasap
