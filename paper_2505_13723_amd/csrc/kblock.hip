// Kernel-block products on the vector ALUs (float64 and float32 arithmetic).
//
// OUT = k(Xr, Xc) R for the column-block oracle K_{B,:} Z (Alg. 2 Step I), the row-block
// sketch K_BB Omega (Step II), the powering matvecs K_BB v (Alg. GetStepsize), residuals
// and predictions.  The b x n kernel block is never stored: each workgroup owns 256 rows
// (one per thread, coordinates in registers), streams a range of columns through LDS in
// tiles of 64 (coordinates and right-hand-side values), evaluates k(x_i, x_j) from
// coordinate differences and accumulates KC right-hand-side columns in registers.  The
// column range is split over gridDim.y workgroups; partial results are summed in a fixed
// order by a second kernel that also applies the epilogue, so results are deterministic.
#include <climits>
#include <cmath>
#include <mutex>
#include <string>

#include "internal.h"
#include "kfun.h"

namespace adasap {

namespace {

constexpr int KB_ROWS = 256;  // rows per workgroup (one per thread)
constexpr int KB_BN = 64;     // columns per LDS tile

template <typename TA>
__device__ inline TA load_as(const void* p, DT t, int64_t i) {
  switch (t) {
    case DT::F64: return TA(static_cast<const double*>(p)[i]);
    case DT::F32: return TA(static_cast<const float*>(p)[i]);
    default: return TA(static_cast<float>(static_cast<const _Float16*>(p)[i]));
  }
}

__device__ inline double load_d(const void* p, DT t, int64_t i) { return load_as<double>(p, t, i); }

template <typename TA, int KERN, int DMAX, int KC>
__global__ __launch_bounds__(KB_ROWS) void kblock_valu_kernel(
    const void* __restrict__ Xr, const int64_t* __restrict__ ridx, DT xt, int64_t m,
    const void* __restrict__ Xc, int64_t n, int d, const void* __restrict__ R, DT rt, int64_t ldr,
    int k, TA* __restrict__ part, int64_t cols_per_split, TA p) {
  __shared__ TA xs[KB_BN * DMAX];
  __shared__ TA rs[KB_BN * KC];
  const int tid = threadIdx.x;
  const int64_t row = (int64_t)blockIdx.x * KB_ROWS + tid;
  const int split = blockIdx.y;
  const int kc0 = blockIdx.z * KC;
  const int64_t c0 = (int64_t)split * cols_per_split;
  const int64_t c1 = c0 + cols_per_split < n ? c0 + cols_per_split : n;
  const bool valid = row < m;
  const int64_t src = valid ? (ridx ? ridx[row] : row) : 0;
  TA xr[DMAX];
#pragma unroll
  for (int f = 0; f < DMAX; ++f) xr[f] = (valid && f < d) ? load_as<TA>(Xr, xt, src * d + f) : TA(0);
  TA acc[KC];
#pragma unroll
  for (int c = 0; c < KC; ++c) acc[c] = TA(0);

  for (int64_t j0 = c0; j0 < c1; j0 += KB_BN) {
    const int nb = (int)((c1 - j0) < KB_BN ? (c1 - j0) : KB_BN);
    for (int e = tid; e < KB_BN * DMAX; e += KB_ROWS) {
      const int j = e / DMAX, f = e % DMAX;
      xs[e] = (j < nb && f < d) ? load_as<TA>(Xc, xt, (j0 + j) * d + f) : TA(0);
    }
    for (int e = tid; e < KB_BN * KC; e += KB_ROWS) {
      const int j = e / KC, c = e % KC;
      rs[e] = (j < nb && kc0 + c < k) ? load_as<TA>(R, rt, (j0 + j) * ldr + kc0 + c) : TA(0);
    }
    __syncthreads();
    for (int j = 0; j < nb; ++j) {
      TA r2 = TA(0);
#pragma unroll
      for (int f = 0; f < DMAX; ++f) {
        const TA df = xr[f] - xs[j * DMAX + f];
        r2 += df * df;
      }
      const TA kv = kfun<KERN, TA>(r2, p);
#pragma unroll
      for (int c = 0; c < KC; ++c) acc[c] += kv * rs[j * KC + c];
    }
    __syncthreads();
  }
  if (valid) {
#pragma unroll
    for (int c = 0; c < KC; ++c)
      if (kc0 + c < k) part[((int64_t)split * m + row) * k + kc0 + c] = acc[c];
  }
}

template <typename TA>
__global__ void kblock_reduce_kernel(const TA* __restrict__ part, int splits, int64_t m, int k,
                                     KbEpilogue ep, void* __restrict__ out, DT ot, int64_t ldo) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= m * k) return;
  const int64_t i = e / k;
  const int c = (int)(e % k);
  double s = 0.0;
  for (int sp = 0; sp < splits; ++sp) s += (double)part[((int64_t)sp * m + i) * k + c];
  s *= ep.kscale;
  if (ep.E1) s += ep.a1 * load_d(ep.E1, ep.e1t, (ep.e1idx ? ep.e1idx[i] : i) * ep.lde1 + c);
  if (ep.E2) s += ep.a2 * load_d(ep.E2, ep.e2t, (ep.e2idx ? ep.e2idx[i] : i) * ep.lde2 + c);
  if (ot == DT::F64) static_cast<double*>(out)[i * ldo + c] = s;
  else static_cast<float*>(out)[i * ldo + c] = (float)s;
}

// per-column sums of squares of a rows x k array: partials per block of rows, then a
// fixed-order sum (deterministic)
constexpr int CN_ROWS = 1024;
__global__ void colsq_partial_kernel(const void* __restrict__ a, DT t, int64_t rows, int k,
                                     int64_t lda, double* __restrict__ part) {
  // one block per CN_ROWS rows; thread c < k sums its column over those rows
  const int64_t r0 = (int64_t)blockIdx.x * CN_ROWS;
  const int64_t r1 = r0 + CN_ROWS < rows ? r0 + CN_ROWS : rows;
  for (int c = threadIdx.x; c < k; c += blockDim.x) {
    double s = 0.0;
    for (int64_t r = r0; r < r1; ++r) {
      const double v = load_d(a, t, r * lda + c);
      s += v * v;
    }
    part[(int64_t)blockIdx.x * k + c] = s;
  }
}

__global__ void colsq_final_kernel(const double* __restrict__ part, int nblk, int k,
                                   double* __restrict__ out) {
  for (int c = threadIdx.x; c < k; c += blockDim.x) {
    double s = 0.0;
    for (int b = 0; b < nblk; ++b) s += part[(int64_t)b * k + c];
    out[c] = s;
  }
}

// Sums over the rows of two rows x k float64 arrays A and C (row i: a_i = |A_i|^2,
// c_i = |C_i|^2): {sum a, sum c, sum a^2, sum c^2, sum a c}, per block of CN_ROWS rows, then
// added in a fixed order (deterministic).
__global__ __launch_bounds__(256) void ratio_stats_partial_kernel(const double* __restrict__ A,
                                                                  const double* __restrict__ C,
                                                                  int64_t rows, int k,
                                                                  double* __restrict__ part) {
  __shared__ double red[5][256];
  const int64_t r0 = (int64_t)blockIdx.x * CN_ROWS;
  const int64_t r1 = r0 + CN_ROWS < rows ? r0 + CN_ROWS : rows;
  double s[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  for (int64_t r = r0 + threadIdx.x; r < r1; r += 256) {
    double a = 0.0, c = 0.0;
    for (int j = 0; j < k; ++j) {
      const double x = A[r * k + j], y = C[r * k + j];
      a += x * x;
      c += y * y;
    }
    s[0] += a;
    s[1] += c;
    s[2] += a * a;
    s[3] += c * c;
    s[4] += a * c;
  }
  for (int q = 0; q < 5; ++q) red[q][threadIdx.x] = s[q];
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h)
      for (int q = 0; q < 5; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x < 5) part[(int64_t)blockIdx.x * 5 + threadIdx.x] = red[threadIdx.x][0];
}

__global__ void ratio_stats_final_kernel(const double* __restrict__ part, int nblk,
                                         double* __restrict__ out) {
  if (threadIdx.x < 5) {
    double s = 0.0;
    for (int b = 0; b < nblk; ++b) s += part[(int64_t)b * 5 + threadIdx.x];
    out[threadIdx.x] = s;
  }
}

template <typename TA, int KERN, int DMAX, int KC>
void launch_valu(dim3 grid, hipStream_t s, const void* Xr, const int64_t* ridx, DT xt, int64_t m,
                 const void* Xc, int64_t n, int d, const void* R, DT rt, int64_t ldr, int k,
                 TA* part, int64_t cps, TA p) {
  hipLaunchKernelGGL((kblock_valu_kernel<TA, KERN, DMAX, KC>), grid, dim3(KB_ROWS), 0, s, Xr,
                     ridx, xt, m, Xc, n, d, R, rt, ldr, k, part, cps, p);
}

template <typename TA, int KERN, int DMAX>
void dispatch_kc(int kc, dim3 grid, hipStream_t s, const void* Xr, const int64_t* ridx, DT xt,
                 int64_t m, const void* Xc, int64_t n, int d, const void* R, DT rt, int64_t ldr,
                 int k, TA* part, int64_t cps, TA p) {
  if (kc == 1) launch_valu<TA, KERN, DMAX, 1>(grid, s, Xr, ridx, xt, m, Xc, n, d, R, rt, ldr, k, part, cps, p);
  else if (kc == 4) launch_valu<TA, KERN, DMAX, 4>(grid, s, Xr, ridx, xt, m, Xc, n, d, R, rt, ldr, k, part, cps, p);
  else launch_valu<TA, KERN, DMAX, 16>(grid, s, Xr, ridx, xt, m, Xc, n, d, R, rt, ldr, k, part, cps, p);
}

template <typename TA, int KERN>
void dispatch_d(int dmax, int kc, dim3 grid, hipStream_t s, const void* Xr, const int64_t* ridx,
                DT xt, int64_t m, const void* Xc, int64_t n, int d, const void* R, DT rt,
                int64_t ldr, int k, TA* part, int64_t cps, TA p) {
  if (dmax == 16) dispatch_kc<TA, KERN, 16>(kc, grid, s, Xr, ridx, xt, m, Xc, n, d, R, rt, ldr, k, part, cps, p);
  else dispatch_kc<TA, KERN, 64>(kc, grid, s, Xr, ridx, xt, m, Xc, n, d, R, rt, ldr, k, part, cps, p);
}

template <typename TA>
void dispatch_kern(int kern, int dmax, int kc, dim3 grid, hipStream_t s, const void* Xr,
                   const int64_t* ridx, DT xt, int64_t m, const void* Xc, int64_t n, int d,
                   const void* R, DT rt, int64_t ldr, int k, TA* part, int64_t cps, TA p) {
  switch (kern) {
    case ADASAP_RBF: dispatch_d<TA, ADASAP_RBF>(dmax, kc, grid, s, Xr, ridx, xt, m, Xc, n, d, R, rt, ldr, k, part, cps, p); break;
    case ADASAP_MATERN12: dispatch_d<TA, ADASAP_MATERN12>(dmax, kc, grid, s, Xr, ridx, xt, m, Xc, n, d, R, rt, ldr, k, part, cps, p); break;
    case ADASAP_MATERN32: dispatch_d<TA, ADASAP_MATERN32>(dmax, kc, grid, s, Xr, ridx, xt, m, Xc, n, d, R, rt, ldr, k, part, cps, p); break;
    default: dispatch_d<TA, ADASAP_MATERN52>(dmax, kc, grid, s, Xr, ridx, xt, m, Xc, n, d, R, rt, ldr, k, part, cps, p); break;
  }
}

}  // namespace

adasap_status_t colsq(int64_t rows, int k, const void* a, DT t, int64_t lda, double* out,
                      DevBuf& tmp, hipStream_t s) {
  const int nblk = (int)((rows + CN_ROWS - 1) / CN_ROWS);
  ADASAP_TRY(tmp.ensure((size_t)(nblk > 0 ? nblk : 1) * k * sizeof(double)));
  if (nblk > 0) {
    hipLaunchKernelGGL(colsq_partial_kernel, dim3(nblk), dim3(128), 0, s, a, t, rows, k, lda,
                       tmp.as<double>());
    ADASAP_LAUNCH_CHECK();
  }
  hipLaunchKernelGGL(colsq_final_kernel, dim3(1), dim3(128), 0, s, tmp.as<double>(), nblk, k, out);
  ADASAP_LAUNCH_CHECK();
  return ADASAP_OK;
}

adasap_status_t ratio_stats(int64_t rows, int k, const double* A, const double* C, double* out,
                            DevBuf& tmp, hipStream_t s) {
  const int nblk = (int)((rows + CN_ROWS - 1) / CN_ROWS);
  ADASAP_TRY(tmp.ensure((size_t)(nblk > 0 ? nblk : 1) * 5 * sizeof(double)));
  if (nblk > 0) {
    hipLaunchKernelGGL(ratio_stats_partial_kernel, dim3(nblk), dim3(256), 0, s, A, C, rows, k,
                       tmp.as<double>());
    ADASAP_LAUNCH_CHECK();
  }
  hipLaunchKernelGGL(ratio_stats_final_kernel, dim3(1), dim3(64), 0, s, tmp.as<double>(), nblk, out);
  ADASAP_LAUNCH_CHECK();
  return ADASAP_OK;
}

namespace {

// Launch plan of a kernel-block product: workgroups of KB_ROWS rows (gx), right-hand-side
// groups of kc columns (gz) and column splits of cps columns.  Enough workgroups to fill 256
// CUs several times, at least one tile per split, and at most max_splits splits.
struct KbPlan {
  int dmax, kc;
  int64_t gx, gz, splits, cps;
};

KbPlan kb_plan(int64_t m, int64_t n, int d, int k, int64_t max_splits) {
  KbPlan pl;
  pl.dmax = d <= 16 ? 16 : 64;
  pl.kc = k == 1 ? 1 : (k <= 4 ? 4 : 16);
  pl.gx = (m + KB_ROWS - 1) / KB_ROWS;
  pl.gz = (k + pl.kc - 1) / pl.kc;
  pl.splits = 0;
  pl.cps = KB_BN;
  if (n > 0) {
    int64_t sp = (2048 + pl.gx * pl.gz - 1) / (pl.gx * pl.gz);
    const int64_t tiles = (n + KB_BN - 1) / KB_BN;
    if (sp > tiles) sp = tiles;
    if (sp > max_splits) sp = max_splits;
    if (sp < 1) sp = 1;
    pl.cps = (n + sp - 1) / sp;
    pl.cps = (pl.cps + KB_BN - 1) / KB_BN * KB_BN;
    pl.splits = (n + pl.cps - 1) / pl.cps;
  }
  return pl;
}

// the product into `part` (splits x m x k of the arithmetic type) and the fixed-order
// reduction with the epilogue; allocates nothing
adasap_status_t kb_launch(const KbPlan& pl, int kern, double ell, int prec, int64_t m, int64_t n,
                          int d, int k, const void* Xr, const int64_t* ridx, DT xt, const void* Xc,
                          const void* R, DT rt, int64_t ldr, void* out, DT ot, int64_t ldo,
                          const KbEpilogue& ep, void* part, hipStream_t s) {
  if (pl.splits > 0) {
    const dim3 grid((unsigned)pl.gx, (unsigned)pl.splits, (unsigned)pl.gz);
    if (prec == ADASAP_FP64)
      dispatch_kern<double>(kern, pl.dmax, pl.kc, grid, s, Xr, ridx, xt, m, Xc, n, d, R, rt, ldr,
                            k, static_cast<double*>(part), pl.cps, kernel_param(kern, ell));
    else
      dispatch_kern<float>(kern, pl.dmax, pl.kc, grid, s, Xr, ridx, xt, m, Xc, n, d, R, rt, ldr, k,
                           static_cast<float*>(part), pl.cps, (float)kernel_param(kern, ell));
    ADASAP_LAUNCH_CHECK();
  }
  // no columns: zero splits, so the reduction writes the epilogue alone
  const unsigned rb = (unsigned)((m * k + 255) / 256);
  if (prec == ADASAP_FP64)
    hipLaunchKernelGGL(kblock_reduce_kernel<double>, dim3(rb), dim3(256), 0, s,
                       static_cast<const double*>(part), (int)pl.splits, m, k, ep, out, ot, ldo);
  else
    hipLaunchKernelGGL(kblock_reduce_kernel<float>, dim3(rb), dim3(256), 0, s,
                       static_cast<const float*>(part), (int)pl.splits, m, k, ep, out, ot, ldo);
  ADASAP_LAUNCH_CHECK();
  return ADASAP_OK;
}

}  // namespace

adasap_status_t kblock_valu(int kern, double ell, int prec, int64_t m, int64_t n, int d, int k,
                            const void* Xr, const int64_t* ridx, DT xt, const void* Xc,
                            const void* R, DT rt, int64_t ldr, void* out, DT ot, int64_t ldo,
                            const KbEpilogue& ep, DevBuf& part, hipStream_t s) {
  if (m <= 0 || k <= 0) return ADASAP_OK;
  if (d < 1 || d > 64) {
    set_error("kblock_valu: d must be in [1, 64]");
    return ADASAP_ERR_INVALID_ARG;
  }
  const KbPlan pl = kb_plan(m, n, d, k, INT64_MAX);
  const size_t tsz = prec == ADASAP_FP64 ? 8 : 4;
  ADASAP_TRY(part.ensure((size_t)(pl.splits > 0 ? pl.splits : 1) * m * k * tsz));
  return kb_launch(pl, kern, ell, prec, m, n, d, k, Xr, ridx, xt, Xc, R, rt, ldr, out, ot, ldo, ep,
                   part.p, s);
}

// ---- the kernel-block product with no allocation ---------------------------------------------
// The split partial sums live in this file-scope device array.  Host code never uses its name
// as an address: each device's copy is looked up once with hipGetSymbolAddress and that
// pointer is what the kernels receive.
constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)32 << 20;
static __device__ __align__(256) char scratch[NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[MAX_DEVICES] = {};

adasap_status_t scratch_address(void** out) {
  int dev = 0;
  ADASAP_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= MAX_DEVICES) {
    set_error("device index out of range for the fixed scratch table");
    return ADASAP_ERR_DEVICE;
  }
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      set_error(std::string("hipGetSymbolAddress of the fixed scratch failed: ") + hipGetErrorString(e));
      return ADASAP_ERR_DEVICE;
    }
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return ADASAP_OK;
}
}  // namespace

}  // namespace adasap

using namespace adasap;

extern "C" adasap_status_t adasap_kblock_matmul_noalloc(int32_t kernel, double lengthscale,
                                                        int32_t precision, int64_t m, int64_t n,
                                                        int32_t d, int32_t k, const void* Xr,
                                                        const void* Xc, const void* R, void* out,
                                                        int32_t dtype, void* stream) {
  if (kernel < 0 || kernel > 3) {
    set_error("unknown kernel");
    return ADASAP_ERR_INVALID_ARG;
  }
  if (!(lengthscale > 0) || !std::isfinite(lengthscale)) {
    set_error("lengthscale must be finite and > 0");
    return ADASAP_ERR_INVALID_ARG;
  }
  if (precision != ADASAP_FP64 && precision != ADASAP_FP32) {
    set_error("the no-allocation product runs in FP64 or FP32 precision");
    return ADASAP_ERR_INVALID_ARG;
  }
  if (m < 0 || n < 0 || d < 1 || d > 64 || k < 1 || k > 128) {
    set_error("need m, n >= 0, 1 <= d <= 64 and 1 <= k <= 128");
    return ADASAP_ERR_INVALID_ARG;
  }
  if (dtype != ADASAP_DTYPE_F32 && dtype != ADASAP_DTYPE_F64) {
    set_error("unknown dtype");
    return ADASAP_ERR_INVALID_ARG;
  }
  const size_t tsz = precision == ADASAP_FP64 ? 8 : 4;
  if ((size_t)m * (size_t)k * tsz > NOALLOC_SCRATCH_BYTES) {
    set_error("m * k * element size exceeds the fixed scratch of " +
              std::to_string(NOALLOC_SCRATCH_BYTES) + " bytes");
    return ADASAP_ERR_INVALID_ARG;
  }
  if (m == 0) return ADASAP_OK;
  if (!Xr || !out || (n > 0 && (!Xc || !R))) {
    set_error("null device pointer");
    return ADASAP_ERR_INVALID_ARG;
  }
  void* part = nullptr;
  ADASAP_TRY(scratch_address(&part));
  const int64_t fit = (int64_t)(NOALLOC_SCRATCH_BYTES / ((size_t)m * k * tsz));
  const KbPlan pl = kb_plan(m, n, d, k, fit);
  const DT t = dtype == ADASAP_DTYPE_F64 ? DT::F64 : DT::F32;
  KbEpilogue none;
  return kb_launch(pl, kernel, lengthscale, precision, m, n, d, k, Xr, nullptr, t, Xc, R, t, k, out,
                   t, k, none, part, static_cast<hipStream_t>(stream));
}

