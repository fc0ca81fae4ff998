// Internal launchers of the ADASAP library.  All launchers enqueue work on `s` and
// return a status; none synchronises unless its comment says so.
#pragma once

#include <vector>

#include "common.h"

namespace adasap {

// Element types understood by the generic launchers.
enum class DT { F32 = 0, F64 = 1, F16 = 2 };

inline size_t dt_size(DT t) { return t == DT::F64 ? 8 : (t == DT::F32 ? 4 : 2); }

// A growable device buffer owned by a handle (or a temporary owner).
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  adasap_status_t ensure(size_t want);
  void release();
  ~DevBuf() { release(); }
  template <typename T>
  T* as() const { return static_cast<T*>(p); }
};

// A batch of P independent problems of identical shapes.  Operand X of problem p starts at
// X + p * sX elements; the launcher comments name which operand each stride belongs to.
// The default (P = 1, zero strides) is a single problem.  Per-problem scalars live in
// consecutive IterScalars entries (problem p uses sc + p).
struct Batch {
  int P = 1;
  int64_t sA = 0, sB = 0, sC = 0, sD = 0, sE = 0;
};
constexpr int64_t SC_DOUBLES = sizeof(IterScalars) / sizeof(double);

// ---- kernel-block products (kblock.hip) -------------------------------------------------
// OUT[i, c] = sum_j k(Xr[ridx? ridx[i] : i], Xc[j]) R[j, c]  (+ epilogue, see KbEpilogue)
// Xr, Xc element type xt; R element type rt (leading dimension ldr); accumulation in the
// arithmetic `prec` (FP64 or FP32 VALU path).  The sum over j is split into `splits`
// column ranges whose partial results are added in a fixed order (deterministic).
struct KbEpilogue {
  // out = kscale * acc + a1 * E1[e1idx? e1idx[i] : i, c] + a2 * E2[...]; E pointers may be null.
  // kscale is the kernel's output scale (K = kscale * k(X, X)).
  double kscale = 1.0;
  const void* E1 = nullptr;
  DT e1t = DT::F64;
  const int64_t* e1idx = nullptr;
  int64_t lde1 = 0;
  double a1 = 0.0;
  const void* E2 = nullptr;
  DT e2t = DT::F64;
  const int64_t* e2idx = nullptr;
  int64_t lde2 = 0;
  double a2 = 0.0;
  // batches: problem p uses E1 + p*bsE1, E2 + p*bsE2 and index lists + p*bsIdx (elements)
  int64_t bsE1 = 0, bsE2 = 0, bsIdx = 0;
};

adasap_status_t kblock_valu(int kern, double ell, int prec, int64_t m, int64_t n, int d, int k,
                            const void* Xr, const int64_t* ridx, DT xt, const void* Xc,
                            const void* R, DT rt, int64_t ldr, void* out, DT ot, int64_t ldo,
                            const KbEpilogue& ep, DevBuf& part, hipStream_t s);

// ---- dense float64 helpers (linalg.hip) ---------------------------------------------------
// P = A^T B over rows [0, rows): A (rows x p, lda, type at), B (rows x q, ldb, type bt);
// result p x q float64 row-major.  If rowscale != null row c of the result is multiplied by
// rowscale[c].
// Batch strides: sA (A), sB (B), sC (P), sD (rowscale).
adasap_status_t gram(int64_t rows, int p, int q, const void* A, DT at, int64_t lda, const void* B,
                     DT bt, int64_t ldb, double* P, const double* rowscale, DevBuf& part,
                     hipStream_t s, const Batch& bt_ = Batch());

// OUT (rows x q, ldo) = alpha_ptr? (*alpha_ptr) * E : 0  +  (A + (delta_ptr? *delta_ptr : 0) * A2) M
// A, A2: rows x p float64 (lda); M: p x q float64 row-major; E: rows x q float64 (lde).
// If alpha_sqrt_inv is set, the factor applied to E is 1/sqrt(*alpha_ptr) instead of 1/(*alpha_ptr);
// alpha_mode: 0 => factor 1 (E added as is), 1 => 1/(*alpha), 2 => 1/sqrt(*alpha).
// Batch strides: sA (A and A2), sB (M), sC (out), sD (E), sE (delta_ptr and alpha_ptr).
adasap_status_t gemm_rm(int64_t rows, int p, int q, const double* A, const double* A2,
                        const double* delta_ptr, int64_t lda, const double* M, double* out,
                        int64_t ldo, const double* E, int64_t lde, const double* alpha_ptr,
                        int alpha_mode, hipStream_t s, const Batch& bt = Batch());

// Nystrom core (one workgroup): from Mo = Omega^T Ysk and Qo = Omega^T Omega (r x r),
// Delta = eps * tr(Mo); C = sym(Mo) + Delta Qo = R^T R (retry Delta *= 10 up to 5 times);
// writes Rinv = R^{-1} (r x r, upper) and scalars->delta / not_pd / failed.
// Batched over P problems (r x r operands consecutive, sc + p).
adasap_status_t nys_core(int r, const double* Mo, const double* Qo, double eps, double* Rinv,
                         double* Rscratch, IterScalars* sc, hipStream_t s, int P = 1);

// Symmetric eigendecomposition of H (r x r, float64) by cyclic Jacobi with the
// round-robin pairing.  Outputs eigenvalues evals (r, unsorted) and eigenvectors V
// (r x r, columns).  rot_buf must hold jacobi_rot_capacity(r) doubles.
size_t jacobi_rot_capacity(int r);
adasap_status_t jacobi_eig(int r, const double* H, double* evals, double* V, double* rot_buf,
                           IterScalars* sc, hipStream_t s, int P = 1);

// Sort eigenpairs descending, S = max(0, sigma^2 - delta), rho (rule 0: lam + S[r-1],
// rule 1: rho_fixed), T = V[:, perm] diag(1/sigma) (so that U = Bm T), and the Woodbury
// coefficient vectors cinv = 1/(S+rho) - 1/rho, cisq = 1/sqrt(S+rho) - 1/sqrt(rho).
adasap_status_t nys_finalize(int r, const double* evals, const double* V, int rho_rule,
                             double lam, double rho_fixed, double* S, double* T, double* cinv,
                             double* cisq, IterScalars* sc, hipStream_t s, int P = 1);

// coefs = 1/(S+rho) - 1/rho (power 0) or 1/sqrt(S+rho) - 1/sqrt(rho) (power 1); sc->rho = rho
adasap_status_t woodbury_coefs(int r, const double* S, double rho, int power, double* coefs,
                               IterScalars* sc, hipStream_t s);

// Vector helpers for randomized powering, batched over P problems with vectors b apart.
// sc->rq = v.z, sc->vnorm2 = z.z (float64, fixed-order reduction), then v = z / sqrt(z.z);
// if last: sc->lam_hat = sc->rq, sc->eta = 1 / sc->rq.  v may equal z.
adasap_status_t dots_normalize(int64_t b, const double* z, double* v, IterScalars* sc, int last,
                               hipStream_t s, int P = 1);
// One powering step carried as w = P^{-1/2} v: sc->rq = w.u, sc->vnorm2 = u.y with
// u = (K + lambda I) w and y = P^{-1} u (y = u without a preconditioner), then w = y / sqrt(u.y);
// if last: sc->lam_hat = sc->rq, sc->eta = 1 / sc->rq.
adasap_status_t power_step(int64_t b, double* w, const double* u, const double* y, IterScalars* sc,
                           int last, hipStream_t s, int P = 1);
// sc->vnorm2 = v.v then v /= sqrt(v.v)
adasap_status_t normalize_inplace(int64_t b, double* v, IterScalars* sc, DevBuf& part,
                                  hipStream_t s, int P = 1);

// ---- exact block projection (chol.hip) ------------------------------------------------------
// H (b x b float64) = outputscale * k(X_B, X_B) + lam I from the points X[B[i]] (type xt), then
// H = L L^T in place (lower triangle) with the inverses of the diagonal blocks in Linv
// (exact_linv_doubles(b) doubles); sc->eta = 1, sc->rho = lam; a failed pivot sets sc->failed.
size_t exact_linv_doubles(int64_t b);
adasap_status_t exact_factor(int kern, double ell, double outputscale, double lam, int64_t b, int d,
                             const void* X, DT xt, const int64_t* B, double* H, double* Linv,
                             IterScalars* sc, hipStream_t s);
// Y (b x k float64) <- (L L^T)^{-1} Y with the factor of exact_factor
adasap_status_t exact_solve(int64_t b, int k, const double* H, const double* Linv, double* Y,
                            hipStream_t s);

// ---- pathwise conditioning (pathwise.hip) ----------------------------------------------------
// out[i, s] = prior[i, s - 1] + out[i, 0] - out[i, s] for s = 1 .. k-1 (out: m x k)
adasap_status_t pathwise_combine(int64_t m, int k, const void* prior, DT pt, void* out, DT ot,
                                 hipStream_t s);

// ---- random numbers (rng.hip) -------------------------------------------------------------
// Batched over P problems: problem p uses seed + p and writes out + p * count.
// If t_dev is set, the stream counter is t + *t_dev, read from device memory at run time.
adasap_status_t normals_dev(uint64_t seed, uint64_t purpose, uint64_t t, int64_t count,
                            double* out, hipStream_t s, int P = 1, const int64_t* t_dev = nullptr);
void sample_block_host(uint64_t seed, uint64_t purpose, uint64_t t, int64_t n, int64_t b,
                       int64_t* out);
// uniform permutation of [0, m) (Fisher-Yates on the stream (seed, purpose, t))
void permutation_host(uint64_t seed, uint64_t purpose, uint64_t t, int64_t m, int64_t* out);

// ---- gathers / Nesterov (update.hip) ------------------------------------------------------
// dst[i, :] (type dt, cols c) = src[idx[i], :] (type st)
adasap_status_t gather_rows(int64_t rows, int cols, const void* src, DT st, int64_t lds,
                            const int64_t* idx, void* dst, DT dt, int64_t ldd, hipStream_t s);
// elementwise copy / convert of a dense n x k array
adasap_status_t convert(int64_t count, const void* src, DT st, void* dst, DT dt, hipStream_t s);
// out (n x d, float64) = X (type xt) with column j multiplied by scale[j] (device array)
adasap_status_t scale_columns(int64_t n, int d, const void* X, DT xt, const double* scale,
                              double* out, hipStream_t s);

struct NestCoef {
  double beta, gamma, alpha;
  int accel, z_uses_v_next;
};
// Dense part on all rows (state type st): V' = beta V + (1-beta) Z, Z' = alpha*V(')+(1-alpha)Z;
// if Wout: Wout = Z (old) before the update (type wt).
// Batch: row_prob (per row) and coefs (beta, gamma, alpha per problem) select each row's constants.
adasap_status_t nesterov_dense(int64_t count, void* V, void* Z, DT st, const NestCoef& c,
                               void* Wout, DT wt, hipStream_t s, const int32_t* row_prob = nullptr,
                               const double* coefs = nullptr, int k = 1);
// Sparse part on the b block rows: with eta = sc->eta,
//  accel: V[B] -= gamma eta D;  Z[B] -= (alpha gamma + 1 - alpha) eta D  (z_uses_v_next)
//                               Z[B] -= (1 - alpha) eta D                 (otherwise)
//         Wout[B] -= eta D if Wout
//  plain: Z[B] -= eta D (Z is the iterate W; V unused)
// Batch: P problems, B and D of problem p at B + p*b, D + p*b*k (B holds global row indices),
// scalars sc + p, constants coefs[3p..3p+2] when coefs is set.
adasap_status_t nesterov_sparse(int64_t b, int k, const int64_t* B, const double* D, void* V,
                                void* Z, DT st, const NestCoef& c, const IterScalars* sc,
                                void* Wout, DT wt, hipStream_t s, int P = 1,
                                const double* coefs = nullptr);
// a += b elementwise (a in place)
adasap_status_t add_inplace(int64_t count, void* a, DT at, const void* b, DT bt, hipStream_t s);
// acc += W (float64 accumulator, count elements) for tail averaging
adasap_status_t accumulate(int64_t count, const void* W, DT wt, double* acc, hipStream_t s);
// dst (type dt) = scale * src (float64)
adasap_status_t scale_store(int64_t count, const double* src, double scale, void* dst, DT dt,
                            hipStream_t s);
// nonzero flag (host int) if any element of src is not finite (synchronises)
adasap_status_t any_nonfinite(int64_t count, const void* src, DT st, int* flag, DevBuf& tmp,
                              hipStream_t s);

}  // namespace adasap
