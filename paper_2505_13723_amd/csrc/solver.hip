// The ADASAP iteration (Alg. 2) on one GPU: handle, workspace, the per-iteration
// sequence of kernels, residual checks, refinement sweeps, prediction.
//
// One iteration t (Sec. 4.2):
//   Step I    B_t sampled on the host (Floyd), copied to the device;
//             G = K(X_B, X) Z_t + lambda Z_t[B] - Y_B               (kernel-block product)
//   Step II   Omega ~ N(0,1)^{b x r} (device Philox), Y_sk = K_BB Omega
//   Step III  Nystrom: Mo = Omega^T Y_sk, Qo = Omega^T Omega, Cholesky of
//             sym(Mo) + Delta Qo, B = (Y_sk + Delta Omega) R^{-1}, Jacobi eigenpairs of
//             B^T B, U = B V Sigma^{-1}, S = max(0, Sigma^2 - Delta), rho;
//             eta = 1 / Rayleigh quotient of 10 powering steps on P^{-1/2}(K_BB+lambda I)P^{-1/2}
//   Step IV   D = P^{-1} G (Woodbury), Nesterov update of (V, Z) (W only when needed)
// All scalars of an iteration stay on the device; the host only launches kernels.
#include <chrono>
#include <cmath>
#include <cstring>
#include <mutex>
#include <vector>

#include "internal.h"
#include "mfma.h"

namespace adasap {

adasap_status_t colsq(int64_t rows, int k, const void* a, DT t, int64_t lda, double* out,
                      DevBuf& tmp, hipStream_t s);
adasap_status_t ratio_stats(int64_t rows, int k, const double* A, const double* C, double* out,
                            DevBuf& tmp, hipStream_t s);

adasap_status_t DevBuf::ensure(size_t want) {
  if (want <= bytes && p) return ADASAP_OK;
  release();
  if (want == 0) want = 16;
  if (hipMalloc(&p, want) != hipSuccess) {
    p = nullptr;
    bytes = 0;
    (void)hipGetLastError();
    set_error("device allocation of " + std::to_string(want) + " bytes failed");
    return ADASAP_ERR_OOM;
  }
  bytes = want;
  return ADASAP_OK;
}

void DevBuf::release() {
  if (p) (void)hipFree(p);
  p = nullptr;
  bytes = 0;
}

}  // namespace adasap

using namespace adasap;

struct adasap_handle_s {
  adasap_config_t cfg;
  int64_t n = 0;
  int d = 0, k = 0;
  DT dtype = DT::F32;  // X, Y, W, predictions
  DT st = DT::F32;     // iterate state V, Z
  hipStream_t s = nullptr;
  const void* X = nullptr;
  const void* Y = nullptr;
  // coordinates every kernel value is computed from: X itself, or with per-coordinate
  // lengthscales the owned float64 copy Xs (coordinate j divided by ell_j) at lengthscale 1
  const void* Xk = nullptr;
  DT xkt = DT::F32;
  double ellk = 1.0;
  std::vector<double> inv_ell;  // 1/ell_j (per-coordinate lengthscales only)
  DevBuf Xs, Xq, iell;          // the scaled copy; scaled prediction points; 1/ell_j (device)
  double mu = 0, nu = 0;
  NestCoef nc{};
  bool use_mfma = false;
  MfmaPack pack;  // packed coordinates for the matrix-core kernel
  // workspace
  DevBuf V, Z, Bdev, XB, G, D, Om, Ysk, Mo, Qo, Rinv, H, evals, Vr, T, S, cinv, cisq, Bm, U, rot;
  DevBuf Hx, Linv;  // exact block projection: factor of K_BB + lambda I, diagonal-block inverses
  DevBuf vv, ww, uu, zz, coef, part_kb, part_g, part_d, scb, tail, res, rhs, delta_w, tmp, colq;
  MfmaWork mw;    // matrix-core scratch of the main stream
  // MIXED accelerated solves: the Nesterov update packs the next Z for Step I in the same pass
  bool fused = false;
  FusedUpd fu;
  MfmaWork mw2;   // matrix-core scratch of the second stream (sketch, powering)
  DevBuf part_kb2, part_g2, coef2;  // second-stream scratch
  hipStream_t s2 = nullptr;         // second stream (default priority)
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  hipEvent_t ev_sketch = nullptr;   // the sketch of the current block is complete
  hipEvent_t ev_bup = nullptr;      // the current block's indices are on the device
  DevBuf Bslot[2];                  // device indices of the blocks of iterations t and t + 1
  int64_t head_t = -1;              // iteration whose head is enqueued on s2 (-1: none)
  uint64_t head_off = 0;
  DevBuf colsB;   // column fragments of the current block
  DevBuf rowq;    // row vectors of prediction points
  int64_t* Bhost[2] = {nullptr, nullptr};
  hipEvent_t bev[2] = {nullptr, nullptr};
  IterScalars* sc_host = nullptr;  // pinned trace of per-iteration scalars
  int64_t sc_host_cap = 0;
  std::vector<double> eta_tr, rho_tr, lh_tr;
  // iterations of the last plain solve whose state (V, Z) the handle still holds, so that
  // adasap_solve_more can continue it (-1: nothing to continue)
  int64_t t_done = -1;
  // ring of event pairs around the step-I product kernel; a pair is read back (long after it
  // completed) when the ring wraps, so no event is created inside the iteration loop
  static constexpr int KEV_RING = 32;
  std::vector<hipEvent_t> kev;
  int64_t kev_used = 0;
  double step1_ms = 0;
  ~adasap_handle_s() {
    for (hipEvent_t e : kev) (void)hipEventDestroy(e);
    if (ev_fork) (void)hipEventDestroy(ev_fork);
    if (ev_join) (void)hipEventDestroy(ev_join);
    if (ev_sketch) (void)hipEventDestroy(ev_sketch);
    if (ev_bup) (void)hipEventDestroy(ev_bup);
    if (s2) (void)hipStreamDestroy(s2);
    for (int i = 0; i < 2; ++i) {
      if (Bhost[i]) (void)hipHostFree(Bhost[i]);
      if (bev[i]) (void)hipEventDestroy(bev[i]);
    }
    if (sc_host) (void)hipHostFree(sc_host);
  }
};

namespace {

thread_local std::string g_last_error;

bool finite_pos(double x) { return std::isfinite(x) && x > 0; }

adasap_status_t invalid(const std::string& m) {
  set_error(m);
  return ADASAP_ERR_INVALID_ARG;
}

adasap_status_t validate(const adasap_config_t* c, int64_t n, int d, int k) {
  if (!c) return invalid("config is null");
  if (c->struct_size != sizeof(adasap_config_t)) return invalid("config struct_size mismatch");
  if (c->kernel < 0 || c->kernel > 3) return invalid("unknown kernel");
  if (c->n_lengthscale != 0 && c->n_lengthscale != 1 && c->n_lengthscale != d)
    return invalid("n_lengthscale must be 0, 1 or d");
  if (c->n_lengthscale == d && d > 1) {
    if (!c->lengthscales) return invalid("lengthscales must be a host array of d entries");
    for (int j = 0; j < d; ++j)
      if (!finite_pos(c->lengthscales[j])) return invalid("lengthscales must be finite and > 0");
  } else if (!finite_pos(c->lengthscale)) {
    return invalid("lengthscale must be finite and > 0");
  }
  if (!finite_pos(c->outputscale)) return invalid("outputscale must be finite and > 0");
  if (c->check_rows < 0) return invalid("check_rows must be >= 0");
  if (!finite_pos(c->lambda)) return invalid("lambda must be finite and > 0");
  if (n < 1) return invalid("n must be >= 1");
  if (d < 1 || d > 64) return invalid("d must be in [1, 64]");
  if (k < 1 || k > 128) return invalid("k must be in [1, 128]");
  if (c->block_size < 1 || c->block_size > n) return invalid("block size must be in [1, n]");
  if (c->precond != ADASAP_PRECOND_NYSTROM && c->precond != ADASAP_PRECOND_IDENTITY &&
      c->precond != ADASAP_PRECOND_EXACT)
    return invalid("unknown preconditioner");
  if (c->precond == ADASAP_PRECOND_EXACT && c->block_size > 16384)
    return invalid("the exact block projection needs b <= 16384 (a b x b float64 factor)");
  if (c->precond == ADASAP_PRECOND_EXACT && c->precision == ADASAP_MIXED)
    return invalid("the exact block projection runs with FP64 or FP32 products (its unit step "
                   "amplifies the float16 error of MIXED products by up to 1/lambda)");
  if (c->precond == ADASAP_PRECOND_NYSTROM &&
      (c->rank < 1 || c->rank > 128 || c->rank > c->block_size))
    return invalid("rank must be in [1, min(b, 128)]");
  if (c->rho_rule != 0 && c->rho_rule != 1) return invalid("rho_rule must be 0 or 1");
  if (c->rho_rule == 1 && !finite_pos(c->rho)) return invalid("rho must be finite and > 0");
  if (c->precision < 0 || c->precision > 2) return invalid("unknown precision");
  if (c->precision == ADASAP_MIXED && d > 16) return invalid("MIXED precision needs d <= 16");
  if (c->precision == ADASAP_MIXED && c->accel && !c->grad_at_z)
    return invalid("MIXED precision evaluates the gradient at Z (grad_at_z = 1)");
  if (c->power_iters < 1 || c->power_iters > 1000) return invalid("power_iters must be in [1, 1000]");
  if (c->max_iters < 0) return invalid("max_iters must be >= 0");
  if (!(c->tol >= 0) || !std::isfinite(c->tol)) return invalid("tol must be finite and >= 0");
  if (c->check_every < 0) return invalid("check_every must be >= 0");
  if (c->refine_sweeps < 0 || c->refine_sweeps > 16) return invalid("refine_sweeps must be in [0, 16]");
  const double mu = c->mu > 0 ? c->mu : c->lambda;
  const double nu = c->nu > 0 ? c->nu : (double)n / (double)c->block_size;
  if (!std::isfinite(mu) || !std::isfinite(nu)) return invalid("mu and nu must be finite");
  if (c->accel && mu > nu) return invalid("need mu <= nu (beta >= 0)");
  return ADASAP_OK;
}

DT to_dt(int32_t dtype) { return dtype == ADASAP_DTYPE_F64 ? DT::F64 : DT::F32; }

double sketch_eps(int prec) { return prec == ADASAP_FP64 ? std::ldexp(1.0, -52) : std::ldexp(1.0, -23); }

// K(rows, cols) R with the handle's precision and kernel
adasap_status_t hk_kblock(adasap_handle_t h, int64_t m, int64_t n, const void* Xr,
                          const int64_t* ridx, DT xt, const void* Xc, const void* R, DT rt,
                          int64_t ldr, int kk, void* out, DT ot, int64_t ldo, const KbEpilogue& ep,
                          int prec, hipStream_t st, DevBuf& part) {
  KbEpilogue e = ep;
  e.kscale = h->cfg.outputscale;
  return kblock_valu(h->cfg.kernel, h->ellk, prec, m, n, h->d, kk, Xr, ridx, xt, Xc, R, rt, ldr, out,
                     ot, ldo, e, part, st);
}

// P^{-1} X (power 0) or P^{-1/2} X (power 1) for the current Nystrom factors; X, out b x kk
adasap_status_t precond_apply_h(adasap_handle_t h, int kk, const double* Xin, double* out,
                                int power, hipStream_t st, DevBuf& part, DevBuf& coef) {
  const int64_t b = h->cfg.block_size;
  const int r = h->cfg.rank;
  IterScalars* sc = h->scb.as<IterScalars>();
  ADASAP_TRY(gram(b, r, kk, h->U.p, DT::F64, r, Xin, DT::F64, kk, coef.as<double>(),
                  power == 0 ? h->cinv.as<double>() : h->cisq.as<double>(), part, st));
  return gemm_rm(b, r, kk, h->U.as<double>(), nullptr, nullptr, r, coef.as<double>(), out, kk,
                 Xin, kk, &sc->rho, power == 0 ? 1 : 2, st);
}

// Step I product G = K(X_B, X) Zc + lambda Zc[B] - rhs[B] (b x k, float64), with the
// launch the solver uses: matrix cores for the reduced precisions (float16 products for
// MIXED, float16 hi/lo or float32-vector products for FP32), vector ALUs otherwise
adasap_status_t block_gradient_h(adasap_handle_t h, const int64_t* B, const void* gp, DT gt,
                                 const void* rhs, DT rhst, double* G, hipStream_t s) {
  const adasap_config_t& c = h->cfg;
  const int64_t n = h->n, b = c.block_size;
  const int k = h->k;
  KbEpilogue epg;
  epg.kscale = c.outputscale;
  epg.E1 = gp;
  epg.e1t = gt;
  epg.e1idx = B;
  epg.lde1 = k;
  epg.a1 = c.lambda;
  epg.E2 = rhs;
  epg.e2t = rhst;
  epg.e2idx = B;
  epg.lde2 = k;
  epg.a2 = -1.0;
  if (h->use_mfma) {
    const int mode = c.precision == ADASAP_MIXED ? mfma_mode_f16()
                                                 : (k <= 4 ? mfma_mode_f32v() : mfma_mode_f16x3());
    return mfma_product(h->pack, B, b, nullptr, 0, gp, gt, k, mode, G, DT::F64, epg, h->mw, s);
  }
  const int kprec = c.precision == ADASAP_FP64 ? ADASAP_FP64 : ADASAP_FP32;
  return hk_kblock(h, b, n, h->Xk, B, h->xkt, h->Xk, gp, gt, k, k, G, DT::F64, k, epg, kprec, s,
                   h->part_kb);
}

// The head of iteration t, on the second stream: the block B_t (host Floyd -> pinned slot ->
// device slot t mod 2), its column fragments (or gathered rows), Omega_t and the sketch
// K_{B_t B_t} Omega_t (Step II).  None of it depends on the iterate, so the previous
// iteration enqueues it behind its own chain, to overlap its update; ev_bup marks the
// indices on the device and ev_sketch the sketch.
adasap_status_t iter_head(adasap_handle_t h, int64_t t, uint64_t off) {
  const adasap_config_t& c = h->cfg;
  const int64_t n = h->n, b = c.block_size;
  const int r = c.rank, d = h->d;
  const int kprec = c.precision == ADASAP_FP64 ? ADASAP_FP64 : ADASAP_FP32;
  hipStream_t s2 = h->s2;
  const int slot = (int)(t & 1);
  ADASAP_HIP(hipEventSynchronize(h->bev[slot]));
  sample_block_host(c.seed, PURPOSE_B + off, (uint64_t)t, n, b, h->Bhost[slot]);
  int64_t* B = h->Bslot[slot].as<int64_t>();
  ADASAP_HIP(hipMemcpyAsync(B, h->Bhost[slot], b * sizeof(int64_t), hipMemcpyHostToDevice, s2));
  ADASAP_HIP(hipEventRecord(h->bev[slot], s2));
  ADASAP_HIP(hipEventRecord(h->ev_bup, s2));
  if (h->use_mfma) ADASAP_TRY(mfma_pack_block(h->pack, B, b, h->colsB, s2));
  else ADASAP_TRY(gather_rows(b, d, h->Xk, h->xkt, d, B, h->XB.p, h->xkt, d, s2));
  if (c.precond == ADASAP_PRECOND_NYSTROM) {
    ADASAP_TRY(normals_dev(c.seed, PURPOSE_OMEGA + off, (uint64_t)t, b * r, h->Om.as<double>(), s2));
    KbEpilogue none;
    none.kscale = c.outputscale;
    if (h->use_mfma)
      ADASAP_TRY(mfma_product(h->pack, B, b, h->colsB.p, b, h->Om.p, DT::F64, r, mfma_mode_f16x3(),
                              h->Ysk.p, DT::F64, none, h->mw2, s2));
    else
      ADASAP_TRY(hk_kblock(h, b, b, h->XB.p, nullptr, h->xkt, h->XB.p, h->Om.p, DT::F64, r, r,
                           h->Ysk.p, DT::F64, r, none, kprec, s2, h->part_kb2));
    ADASAP_HIP(hipEventRecord(h->ev_sketch, s2));
  }
  h->head_t = t;
  h->head_off = off;
  return ADASAP_OK;
}

// one ADASAP iteration; rhs is the current right-hand side (Y or a refinement residual);
// with prefetch_next the head of iteration t + 1 is enqueued behind this iteration's chain
adasap_status_t iterate(adasap_handle_t h, int64_t t, uint64_t off, const void* rhs, DT rhst,
                        void* Wout, bool prefetch_next) {
  const adasap_config_t& c = h->cfg;
  const int64_t n = h->n, b = c.block_size;
  const int k = h->k, r = c.rank;
  hipStream_t s = h->s;
  IterScalars* sc = h->scb.as<IterScalars>();
  const int prec = c.precision;
  const int kprec = prec == ADASAP_FP64 ? ADASAP_FP64 : ADASAP_FP32;
  const bool nys = c.precond == ADASAP_PRECOND_NYSTROM;

  // The sketch, the Nystrom factors and the step size do not depend on the block gradient:
  // they run on a second stream while the main stream evaluates K_{B,:} Z.  That stream
  // rewrites the factors and scalars the previous update read, so it first waits for the
  // main stream's work so far; the head of this iteration (block, sketch) may already be
  // queued before the wait.  The sketch is a matrix-core product that would compete with
  // Step I, so the Step-I product waits for it (the main stream packs Z meanwhile); the rest
  // of the chain, mostly small kernels, runs beside Step I.
  hipStream_t s2 = h->s2;
  ADASAP_HIP(hipEventRecord(h->ev_fork, s));
  ADASAP_HIP(hipStreamWaitEvent(s2, h->ev_fork, 0));
  if (h->head_t != t || h->head_off != off) ADASAP_TRY(iter_head(h, t, off));
  h->head_t = -1;
  const int64_t* B = h->Bslot[t & 1].as<int64_t>();
  ADASAP_HIP(hipStreamWaitEvent(s, h->ev_bup, 0));
  const bool sketch_first = nys && h->use_mfma;

  // gradient block at Z (accelerated; the reading of Alg. 2 Step IV), at W_t (accelerated,
  // printed form) or at the iterate (plain steps keep the iterate in Z)
  const bool at_w = c.accel && !c.grad_at_z;
  const void* gp = at_w ? Wout : h->Z.p;
  const DT gt = at_w ? h->dtype : h->st;
  if (h->use_mfma) {
    const int ring = adasap_handle_s::KEV_RING;
    const bool fz = h->fused && !at_w;
    if (h->kev.empty()) {
      for (int e = 0; e < 2 * ring; ++e) {
        hipEvent_t ev;
        ADASAP_HIP(hipEventCreate(&ev));
        h->kev.push_back(ev);
      }
    }
    const int slot = (int)(h->kev_used % ring);
    if (h->kev_used >= ring) {
      float ms = 0;
      ADASAP_HIP(hipEventSynchronize(h->kev[2 * slot + 1]));
      ADASAP_HIP(hipEventElapsedTime(&ms, h->kev[2 * slot], h->kev[2 * slot + 1]));
      h->step1_ms += ms;
    }
    h->mw.ev0 = h->kev[2 * slot];
    h->mw.ev1 = h->kev[2 * slot + 1];
    h->mw.wait_ev = sketch_first ? h->ev_sketch : nullptr;
    ++h->kev_used;
    adasap_status_t pst;
    if (fz) {
      // Z_t was packed by the previous update (or at the start of the sweep)
      KbEpilogue epg;
      epg.kscale = c.outputscale;
      epg.E1 = gp;
      epg.e1t = gt;
      epg.e1idx = B;
      epg.lde1 = k;
      epg.a1 = c.lambda;
      epg.E2 = rhs;
      epg.e2t = rhst;
      epg.e2idx = B;
      epg.lde2 = k;
      epg.a2 = -1.0;
      pst = mfma_product_packed(h->pack, B, b, fused_rhs(h->fu), k, h->G.p, DT::F64, epg, h->mw, s);
    } else {
      pst = block_gradient_h(h, B, gp, gt, rhs, rhst, h->G.as<double>(), s);
    }
    h->mw.ev0 = h->mw.ev1 = nullptr;
    h->mw.wait_ev = nullptr;
    ADASAP_TRY(pst);
  } else {
    ADASAP_TRY(block_gradient_h(h, B, gp, gt, rhs, rhst, h->G.as<double>(), s));
  }

  const bool exact = c.precond == ADASAP_PRECOND_EXACT;
  if (exact) {
    // Alg. 1: the exact projection onto the block, P_B = K_BB + lambda I, unit step
    ADASAP_TRY(exact_factor(c.kernel, h->ellk, c.outputscale, c.lambda, b, h->d, h->Xk, h->xkt, B,
                            h->Hx.as<double>(), h->Linv.as<double>(), sc, s2));
  }
  if (nys) {
    // Step III: Nystrom factors
    ADASAP_TRY(gram(b, r, r, h->Om.p, DT::F64, r, h->Ysk.p, DT::F64, r, h->Mo.as<double>(), nullptr,
                    h->part_g2, s2));
    ADASAP_TRY(gram(b, r, r, h->Om.p, DT::F64, r, h->Om.p, DT::F64, r, h->Qo.as<double>(), nullptr,
                    h->part_g2, s2));
    ADASAP_TRY(nys_core(r, h->Mo.as<double>(), h->Qo.as<double>(), sketch_eps(prec),
                        h->Rinv.as<double>(), nullptr, sc, s2));
    ADASAP_TRY(gemm_rm(b, r, r, h->Ysk.as<double>(), h->Om.as<double>(), &sc->delta, r,
                       h->Rinv.as<double>(), h->Bm.as<double>(), r, nullptr, 0, nullptr, 0, s2));
    ADASAP_TRY(gram(b, r, r, h->Bm.p, DT::F64, r, h->Bm.p, DT::F64, r, h->H.as<double>(), nullptr,
                    h->part_g2, s2));
    ADASAP_TRY(jacobi_eig(r, h->H.as<double>(), h->evals.as<double>(), h->Vr.as<double>(),
                          h->rot.as<double>(), sc, s2));
    ADASAP_TRY(nys_finalize(r, h->evals.as<double>(), h->Vr.as<double>(), c.rho_rule, c.lambda,
                            c.rho, h->S.as<double>(), h->T.as<double>(), h->cinv.as<double>(),
                            h->cisq.as<double>(), sc, s2));
    ADASAP_TRY(gemm_rm(b, r, r, h->Bm.as<double>(), nullptr, nullptr, r, h->T.as<double>(),
                       h->U.as<double>(), r, nullptr, 0, nullptr, 0, s2));
  }
  // step size by randomized powering (Alg. GetStepsize) on P^{-1/2} (K_BB + lambda I) P^{-1/2},
  // carried as w = P^{-1/2} v: one P^{-1} apply per step (power_step)
  double* v = h->vv.as<double>();
  double* w = h->ww.as<double>();
  double* u = h->uu.as<double>();
  double* z = h->zz.as<double>();
  double* wc = v;
  if (!exact) {
    ADASAP_TRY(normals_dev(c.seed, PURPOSE_POW + off, (uint64_t)t, b, v, s2));
    ADASAP_TRY(normalize_inplace(b, v, sc, h->part_d, s2));
    if (nys) {
      ADASAP_TRY(precond_apply_h(h, 1, v, w, 1, s2, h->part_g2, h->coef2));
      wc = w;
    }
  }
  for (int i = 0; i < (exact ? 0 : c.power_iters); ++i) {
    KbEpilogue epp;
    epp.kscale = c.outputscale;
    epp.E1 = wc;
    epp.e1t = DT::F64;
    epp.lde1 = 1;
    epp.a1 = c.lambda;
    if (h->use_mfma)
      ADASAP_TRY(mfma_product(h->pack, B, b, h->colsB.p, b, wc, DT::F64, 1, mfma_mode_f32v(), u,
                              DT::F64, epp, h->mw2, s2));
    else
      ADASAP_TRY(hk_kblock(h, b, b, h->XB.p, nullptr, h->xkt, h->XB.p, wc, DT::F64, 1, 1, u,
                           DT::F64, 1, epp, kprec, s2, h->part_kb2));
    const double* y = u;
    if (nys) {
      ADASAP_TRY(precond_apply_h(h, 1, u, z, 0, s2, h->part_g2, h->coef2));
      y = z;
    }
    ADASAP_TRY(power_step(b, wc, u, y, sc, i == c.power_iters - 1 ? 1 : 0, s2));
  }
  // join: the direction needs both the block gradient and the Nystrom factors
  ADASAP_HIP(hipEventRecord(h->ev_join, s2));
  ADASAP_HIP(hipStreamWaitEvent(s, h->ev_join, 0));
  // Step IV: direction and update
  const double* Dp = h->G.as<double>();
  if (nys) {
    ADASAP_TRY(precond_apply_h(h, k, h->G.as<double>(), h->D.as<double>(), 0, s, h->part_g, h->coef));
    Dp = h->D.as<double>();
  } else if (exact) {
    ADASAP_HIP(hipMemcpyAsync(h->D.p, h->G.p, (size_t)b * k * sizeof(double), hipMemcpyDeviceToDevice, s));
    ADASAP_TRY(exact_solve(b, k, h->Hx.as<double>(), h->Linv.as<double>(), h->D.as<double>(), s));
    Dp = h->D.as<double>();
  }
  if (h->fused) {
    // all-rows and block-row parts of the update in one pass that also packs Z_{t+1}
    ADASAP_TRY(fused_update(h->pack, h->fu, k, B, b, Dp, sc, h->nc, h->V.as<float>(),
                            h->Z.as<float>(), Wout, h->dtype, s));
  } else {
    if (c.accel) ADASAP_TRY(nesterov_dense(n * k, h->V.p, h->Z.p, h->st, h->nc, Wout, h->dtype, s));
    ADASAP_TRY(nesterov_sparse(b, k, B, Dp, h->V.p, h->Z.p, h->st, h->nc, sc,
                               c.accel ? Wout : nullptr, h->dtype, s));
  }
  // the head of the next iteration (host sampling of B_{t+1}, then its second-stream work)
  // is enqueued after this update, so that the update never waits for the host's sampling
  if (prefetch_next) ADASAP_TRY(iter_head(h, t + 1, off));
  return ADASAP_OK;
}

adasap_status_t residual_h(adasap_handle_t h, const void* W, DT wt, const void* rhs, DT rhst,
                           double* relres, double* relmax, bool keep) {
  const int64_t n = h->n;
  const int k = h->k;
  ADASAP_TRY(h->res.ensure((size_t)n * k * sizeof(double)));
  ADASAP_TRY(h->colq.ensure(2 * (size_t)k * sizeof(double)));
  KbEpilogue ep;
  ep.kscale = h->cfg.outputscale;
  ep.E1 = W;
  ep.e1t = wt;
  ep.lde1 = k;
  ep.a1 = h->cfg.lambda;
  ep.E2 = rhs;
  ep.e2t = rhst;
  ep.lde2 = k;
  ep.a2 = -1.0;
  if (h->use_mfma) {
    // the residual runs alone: the full grid, not the Step-I cap
    const int cap = h->mw.cap_cus;
    h->mw.cap_cus = 0;
    const adasap_status_t pst = mfma_product(h->pack, nullptr, n, nullptr, 0, W, wt, k,
                                             mfma_mode_f16x3(), h->res.p, DT::F64, ep, h->mw, h->s);
    h->mw.cap_cus = cap;
    ADASAP_TRY(pst);
  } else {
    ADASAP_TRY(hk_kblock(h, n, n, h->Xk, nullptr, h->xkt, h->Xk, W, wt, k, k, h->res.p, DT::F64, k,
                         ep, ADASAP_FP64, h->s, h->part_kb));
  }
  double* cq = h->colq.as<double>();
  ADASAP_TRY(colsq(n, k, h->res.p, DT::F64, k, cq, h->tmp, h->s));
  ADASAP_TRY(colsq(n, k, rhs, rhst, k, cq + k, h->tmp, h->s));
  std::vector<double> hq(2 * (size_t)k);
  ADASAP_HIP(hipMemcpyAsync(hq.data(), cq, 2 * (size_t)k * sizeof(double), hipMemcpyDeviceToHost, h->s));
  ADASAP_HIP(hipStreamSynchronize(h->s));
  double rs = 0, ys = 0, mx = 0;
  for (int c = 0; c < k; ++c) {
    rs += hq[c];
    ys += hq[k + c];
    const double col = hq[k + c] > 0 ? std::sqrt(hq[c] / hq[k + c]) : std::sqrt(hq[c]);
    mx = col > mx ? col : mx;
  }
  if (relres) *relres = ys > 0 ? std::sqrt(rs / ys) : std::sqrt(rs);
  if (relmax) *relmax = mx;
  (void)keep;
  return ADASAP_OK;
}

adasap_status_t residual_rows_h(adasap_handle_t h, const void* W, DT wt, const void* rhs, DT rhst,
                                int64_t m, uint64_t seed, bool fp64, double* relres,
                                double* relres_maxcol, double* rel_se, int64_t* rows_out);

// solve (K + lambda I) Wst = rhs from the state already in (V, Z); writes W (handle dtype)
adasap_status_t run_sweep(adasap_handle_t h, uint64_t off, const void* rhs, DT rhst, void* W,
                          int64_t t0, int64_t T, int64_t& iters_done, double& relres,
                          double& relmax, double& solve_ms, double& check_ms,
                          int64_t& trace_pos) {
  const adasap_config_t& c = h->cfg;
  const int64_t nk = h->n * h->k;
  // device time of the iterations: one event pair per segment between residual checks;
  // nothing synchronises inside a segment, so the host samples the next block while the
  // device works
  hipEvent_t e0, e1;
  ADASAP_HIP(hipEventCreate(&e0));
  ADASAP_HIP(hipEventCreate(&e1));
  bool seg_open = false;
  auto close_segment = [&]() -> adasap_status_t {
    if (!seg_open) return ADASAP_OK;
    ADASAP_HIP(hipEventRecord(e1, h->s));
    ADASAP_HIP(hipEventSynchronize(e1));
    float ms = 0;
    ADASAP_HIP(hipEventElapsedTime(&ms, e0, e1));
    solve_ms += ms;
    seg_open = false;
    return ADASAP_OK;
  };
  const bool tail = c.tail_average != 0;
  int64_t tail_count = 0;
  if (tail) {
    ADASAP_TRY(h->tail.ensure((size_t)nk * sizeof(double)));
    ADASAP_HIP(hipMemsetAsync(h->tail.p, 0, (size_t)nk * sizeof(double), h->s));
  }
  const int64_t every = (c.tol > 0) ? (c.check_every > 0 ? c.check_every : T) : 0;
  if (h->fused && T > 0)
    ADASAP_TRY(fused_init(h->pack, h->fu, h->k, h->V.as<float>(), h->Z.as<float>(), h->mw, h->s));
  for (int64_t i = 0; i < T; ++i) {
    const int64_t t = t0 + i;
    if (tail && i >= T / 2) {
      ADASAP_TRY(accumulate(nk, W, h->dtype, h->tail.as<double>(), h->s));
      ++tail_count;
    }
    const bool check_now = every > 0 && ((i + 1) % every == 0 || i + 1 == T);
    const bool need_w = tail || check_now || i + 1 == T || (c.accel && !c.grad_at_z);
    if (!seg_open) {
      ADASAP_HIP(hipEventRecord(e0, h->s));
      seg_open = true;
    }
    ADASAP_TRY(iterate(h, t, off, rhs, rhst, need_w || !c.accel ? W : nullptr, i + 1 < T));
    if (trace_pos < h->sc_host_cap) {
      ADASAP_HIP(hipMemcpyAsync(h->sc_host + trace_pos, h->scb.p, sizeof(IterScalars),
                                hipMemcpyDeviceToHost, h->s));
    }
    ++trace_pos;
    ++iters_done;
    if (!c.accel && need_w) ADASAP_TRY(convert(nk, h->Z.p, h->st, W, h->dtype, h->s));
    if (check_now) {
      ADASAP_TRY(close_segment());
      auto c0 = std::chrono::steady_clock::now();
      if (c.check_rows > 0)
        ADASAP_TRY(residual_rows_h(h, W, h->dtype, rhs, rhst, c.check_rows < h->n ? c.check_rows : h->n,
                                   c.seed, false, &relres, &relmax, nullptr, nullptr));
      else
        ADASAP_TRY(residual_h(h, W, h->dtype, rhs, rhst, &relres, &relmax, false));
      check_ms += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - c0).count();
      if (!std::isfinite(relres)) {
        set_error("non-finite residual");
        (void)hipStreamSynchronize(h->s2);
        h->head_t = -1;
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        return ADASAP_ERR_NONFINITE;
      }
      if (relres <= c.tol) break;
    }
  }
  ADASAP_TRY(close_segment());
  if (!c.accel) ADASAP_TRY(convert(nk, h->Z.p, h->st, W, h->dtype, h->s));
  if (tail && tail_count > 0)
    ADASAP_TRY(scale_store(nk, h->tail.as<double>(), 1.0 / (double)tail_count, W, h->dtype, h->s));
  ADASAP_HIP(hipStreamSynchronize(h->s));
  // a head enqueued for an iteration that did not run (converged) is finished and dropped
  ADASAP_HIP(hipStreamSynchronize(h->s2));
  h->head_t = -1;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return ADASAP_OK;
}

// Row-subsampled relative residual: m rows S (Floyd on (seed, 12, 0)), each computed against
// all n columns with the handle's products (matrix-core hi/lo or float64) or, with fp64, with
// float64 kernel values and products; optionally the relative standard error of the ratio
// estimate (delta method, finite-population corrected).
adasap_status_t residual_rows_h(adasap_handle_t h, const void* W, DT wt, const void* rhs, DT rhst,
                                int64_t m, uint64_t seed, bool fp64, double* relres,
                                double* relres_maxcol, double* rel_se, int64_t* rows_out) {
  if (!h) return invalid("handle is null");
  if (!W) return invalid("W must be a non-null device pointer");
  if (m < 1 || m > h->n) return invalid("m must be in [1, n]");
  const int64_t n = h->n;
  const int k = h->k;
  std::vector<int64_t> rows((size_t)m);
  sample_block_host(seed, PURPOSE_RESROWS, 0, n, m, rows.data());
  DevBuf rdev, yrows, stats;
  ADASAP_TRY(rdev.ensure((size_t)m * sizeof(int64_t)));
  ADASAP_TRY(yrows.ensure((size_t)m * k * sizeof(double)));
  ADASAP_TRY(stats.ensure(5 * sizeof(double)));
  ADASAP_TRY(h->res.ensure((size_t)m * k * sizeof(double)));
  ADASAP_TRY(h->colq.ensure(2 * (size_t)k * sizeof(double)));
  ADASAP_HIP(hipMemcpyAsync(rdev.p, rows.data(), (size_t)m * sizeof(int64_t), hipMemcpyHostToDevice, h->s));
  const int64_t* ridx = rdev.as<int64_t>();
  KbEpilogue ep;
  ep.kscale = h->cfg.outputscale;
  ep.E1 = W;
  ep.e1t = wt;
  ep.e1idx = ridx;
  ep.lde1 = k;
  ep.a1 = h->cfg.lambda;
  ep.E2 = rhs;
  ep.e2t = rhst;
  ep.e2idx = ridx;
  ep.lde2 = k;
  ep.a2 = -1.0;
  if (h->use_mfma && !fp64) {
    const int cap = h->mw.cap_cus;
    h->mw.cap_cus = 0;
    const adasap_status_t pst = mfma_product(h->pack, ridx, m, nullptr, 0, W, wt, k,
                                             mfma_mode_f16x3(), h->res.p, DT::F64, ep, h->mw, h->s);
    h->mw.cap_cus = cap;
    ADASAP_TRY(pst);
  } else {
    ADASAP_TRY(hk_kblock(h, m, n, h->Xk, ridx, h->xkt, h->Xk, W, wt, k, k, h->res.p, DT::F64, k, ep,
                         ADASAP_FP64, h->s, h->part_kb));
  }
  ADASAP_TRY(gather_rows(m, k, rhs, rhst, k, ridx, yrows.p, DT::F64, k, h->s));
  double* cq = h->colq.as<double>();
  ADASAP_TRY(colsq(m, k, h->res.p, DT::F64, k, cq, h->tmp, h->s));
  ADASAP_TRY(colsq(m, k, yrows.p, DT::F64, k, cq + k, h->tmp, h->s));
  std::vector<double> hq(2 * (size_t)k);
  double st[5] = {0, 0, 0, 0, 0};
  ADASAP_HIP(hipMemcpyAsync(hq.data(), cq, 2 * (size_t)k * sizeof(double), hipMemcpyDeviceToHost, h->s));
  if (rel_se) {
    ADASAP_TRY(ratio_stats(m, k, h->res.as<double>(), yrows.as<double>(), stats.as<double>(), h->tmp,
                           h->s));
    ADASAP_HIP(hipMemcpyAsync(st, stats.p, 5 * sizeof(double), hipMemcpyDeviceToHost, h->s));
  }
  if (rows_out)
    ADASAP_HIP(hipMemcpyAsync(rows_out, ridx, (size_t)m * sizeof(int64_t), hipMemcpyDeviceToDevice, h->s));
  ADASAP_HIP(hipStreamSynchronize(h->s));
  double rs = 0, ys = 0, mx = 0;
  for (int c = 0; c < k; ++c) {
    rs += hq[c];
    ys += hq[k + c];
    const double col = hq[k + c] > 0 ? std::sqrt(hq[c] / hq[k + c]) : std::sqrt(hq[c]);
    mx = col > mx ? col : mx;
  }
  if (relres) *relres = ys > 0 ? std::sqrt(rs / ys) : std::sqrt(rs);
  if (relres_maxcol) *relres_maxcol = mx;
  if (rel_se) {
    // Rhat = sum a / sum c; s^2 = sum (a - Rhat c)^2 / (m - 1); Var(Rhat) = (1 - m/n) s^2 / (m cbar^2)
    const double A = st[0], C = st[1];
    double se = 0.0;
    if (m > 1 && A > 0 && C > 0) {
      const double R = A / C;
      const double ss = st[2] - 2.0 * R * st[4] + R * R * st[3];
      const double s2 = (ss > 0 ? ss : 0.0) / (double)(m - 1);
      const double cbar = C / (double)m;
      const double var = (1.0 - (double)m / (double)n) * s2 / ((double)m * cbar * cbar);
      se = 0.5 * std::sqrt(var) / R;
    }
    *rel_se = se;
  }
  return ADASAP_OK;
}

// out (m x k, handle dtype) = K(X*, X) W, enqueued on the handle's stream
adasap_status_t predict_h(adasap_handle_t h, const void* W, int64_t m, const void* Xstar, void* out) {
  KbEpilogue none;
  const int kprec = h->cfg.precision == ADASAP_FP64 ? ADASAP_FP64 : ADASAP_FP32;
  // prediction points in the coordinates the kernel values are computed from
  const void* Xq = Xstar;
  DT xqt = h->dtype;
  if (!h->inv_ell.empty()) {
    ADASAP_TRY(h->Xq.ensure((size_t)m * h->d * 8));
    ADASAP_TRY(scale_columns(m, h->d, Xstar, h->dtype, h->iell.as<double>(), h->Xq.as<double>(), h->s));
    Xq = h->Xq.p;
    xqt = DT::F64;
  }
  if (h->use_mfma) {
    ADASAP_TRY(mfma_points(h->pack, Xq, xqt, m, h->rowq, h->s));
    ADASAP_TRY(mfma_product_rows(h->pack, h->rowq.p, m, W, h->dtype, h->k, mfma_mode_f16x3(), out,
                                 h->dtype, h->mw, h->s, h->cfg.outputscale));
  } else {
    ADASAP_TRY(hk_kblock(h, m, h->n, Xq, nullptr, xqt, h->Xk, W, h->dtype, h->k, h->k, out, h->dtype,
                         h->k, none, kprec, h->s, h->part_kb));
  }
  return ADASAP_OK;
}

// pinned trace of per-iteration scalars for `iters` iterations
adasap_status_t ensure_trace(adasap_handle_t h, int64_t iters) {
  if (h->sc_host_cap >= iters) return ADASAP_OK;
  if (h->sc_host) (void)hipHostFree(h->sc_host);
  h->sc_host = nullptr;
  h->sc_host_cap = 0;
  if (iters > 0) {
    if (hipHostMalloc((void**)&h->sc_host, iters * sizeof(IterScalars)) != hipSuccess) {
      set_error("pinned host allocation failed");
      return ADASAP_ERR_OOM;
    }
    h->sc_host_cap = iters;
  }
  return ADASAP_OK;
}

// fills the report from the per-iteration trace and the timing ring of the finished run
adasap_status_t finish_report(adasap_handle_t h, adasap_report_t& rep, int64_t trace_pos,
                              double relres, double relmax) {
  const adasap_config_t& c = h->cfg;
  ADASAP_HIP(hipStreamSynchronize(h->s));
  const int64_t ntr = trace_pos < h->sc_host_cap ? trace_pos : h->sc_host_cap;
  h->eta_tr.resize(ntr);
  h->rho_tr.resize(ntr);
  h->lh_tr.resize(ntr);
  for (int64_t i = 0; i < ntr; ++i) {
    h->eta_tr[i] = h->sc_host[i].eta;
    h->rho_tr[i] = h->sc_host[i].rho;
    h->lh_tr[i] = h->sc_host[i].lam_hat;
    rep.not_pd_events += h->sc_host[i].not_pd;
    if (h->sc_host[i].sweeps > rep.jacobi_sweeps_max) rep.jacobi_sweeps_max = h->sc_host[i].sweeps;
    if (h->sc_host[i].failed) {
      set_error("Nystrom core not positive definite after shift retries");
      rep.status = ADASAP_ERR_NOT_PD;
    }
  }
  if (ntr > 0) {
    rep.eta_last = h->eta_tr[ntr - 1];
    rep.rho_last = h->rho_tr[ntr - 1];
    rep.lambda_hat_last = h->lh_tr[ntr - 1];
    rep.delta_last = h->sc_host[ntr - 1].delta;
  }
  rep.relres = relres;
  rep.relres_maxcol = relmax;
  {
    const int ring = adasap_handle_s::KEV_RING;
    const int64_t pending = h->kev_used < ring ? h->kev_used : ring;
    rep.step1_kernel_ms = h->step1_ms;
    for (int64_t i = 0; i < pending; ++i) {
      const int slot = (int)((h->kev_used - 1 - i) % ring);
      float ms = 0;
      if (hipEventElapsedTime(&ms, h->kev[2 * slot], h->kev[2 * slot + 1]) == hipSuccess)
        rep.step1_kernel_ms += ms;
    }
  }
  rep.step1_launches = h->kev_used;
  if (rep.status == ADASAP_OK && c.tol > 0 && !(relres >= 0 && relres <= c.tol)) {
    set_error("relative residual " + std::to_string(relres) + " above tol " + std::to_string(c.tol));
    rep.status = ADASAP_ERR_NOT_CONVERGED;
  }
  return ADASAP_OK;
}

}  // namespace

namespace adasap {
void set_error(const std::string& msg) { g_last_error = msg; }
}  // namespace adasap

extern "C" {

adasap_status_t adasap_config_default(adasap_config_t* cfg) {
  if (!cfg) return invalid("config is null");
  std::memset(cfg, 0, sizeof(*cfg));
  cfg->struct_size = sizeof(adasap_config_t);
  cfg->kernel = ADASAP_RBF;
  cfg->lengthscale = 1.0;
  cfg->lambda = 1e-2;
  cfg->block_size = 256;
  cfg->rank = 64;
  cfg->rho_rule = 0;
  cfg->rho = 0.0;
  cfg->mu = 0.0;
  cfg->nu = 0.0;
  cfg->power_iters = 10;
  cfg->max_iters = 100;
  cfg->tol = 0.0;
  cfg->check_every = 0;
  cfg->refine_sweeps = 0;
  cfg->precond = ADASAP_PRECOND_NYSTROM;
  cfg->precision = ADASAP_FP32;
  cfg->seed = 0;
  cfg->accel = 1;
  cfg->grad_at_z = 1;
  cfg->z_uses_v_next = 1;
  cfg->tail_average = 0;
  cfg->n_lengthscale = 0;
  cfg->lengthscales = nullptr;
  cfg->outputscale = 1.0;
  cfg->check_rows = 0;
  return ADASAP_OK;
}

int64_t adasap_workspace_bytes(const adasap_config_t* cfg, int64_t n, int32_t d, int32_t k) {
  if (validate(cfg, n, d, k) != ADASAP_OK) return 0;
  const int64_t b = cfg->block_size, r = cfg->rank;
  const int64_t st = cfg->precision == ADASAP_FP64 ? 8 : 4;
  int64_t bytes = 2 * n * k * st;                       // V, Z
  bytes += b * (8 + 8 * d + 16 * k + 24 * r + 32);      // B, X_B, G, D, Omega, Y_sk, B, U, vectors
  bytes += 8 * r * r * 8 + 8 * (int64_t)jacobi_rot_capacity((int)r);
  if (cfg->precond == ADASAP_PRECOND_EXACT) bytes += b * b * 8 + (int64_t)exact_linv_doubles(b) * 8;
  if (cfg->precision != ADASAP_FP64 && d <= 16) bytes += mfma_pack_bytes(n, d, k);
  if (cfg->n_lengthscale == d && d > 1) bytes += n * d * 8;  // scaled copy of X
  return bytes;
}

adasap_status_t adasap_create(const adasap_config_t* cfg, int64_t n, int32_t d, int32_t k,
                              const void* X, const void* Y, int32_t dtype, void* stream,
                              adasap_handle_t* out) {
  if (!out) return invalid("out handle pointer is null");
  *out = nullptr;
  ADASAP_TRY(validate(cfg, n, d, k));
  if (!X || !Y) return invalid("X and Y must be non-null device pointers");
  if (dtype != ADASAP_DTYPE_F32 && dtype != ADASAP_DTYPE_F64) return invalid("unknown dtype");
  auto* h = new (std::nothrow) adasap_handle_s();
  if (!h) return ADASAP_ERR_OOM;
  h->cfg = *cfg;
  h->n = n;
  h->d = d;
  h->k = k;
  h->dtype = to_dt(dtype);
  h->st = cfg->precision == ADASAP_FP64 ? DT::F64 : DT::F32;
  h->s = static_cast<hipStream_t>(stream);
  h->X = X;
  h->Y = Y;
  h->Xk = X;
  h->xkt = h->dtype;
  h->ellk = cfg->lengthscale;
  h->mu = cfg->mu > 0 ? cfg->mu : cfg->lambda;
  h->nu = cfg->nu > 0 ? cfg->nu : (double)n / (double)cfg->block_size;
  h->nc.beta = 1.0 - std::sqrt(h->mu / h->nu);
  h->nc.gamma = 1.0 / std::sqrt(h->mu * h->nu);
  h->nc.alpha = 1.0 / (1.0 + h->nc.gamma * h->nu);
  h->nc.accel = cfg->accel ? 1 : 0;
  h->nc.z_uses_v_next = cfg->z_uses_v_next ? 1 : 0;
  // matrix-core products for the reduced precisions whenever the coordinates fit them
  h->use_mfma = cfg->precision != ADASAP_FP64 && d <= 16;
  auto fail = [&](adasap_status_t st) {
    delete h;
    return st;
  };
  const int64_t b = cfg->block_size;
  const int r = cfg->rank > 0 ? cfg->rank : 1;
  const size_t ss = dt_size(h->st);
  adasap_status_t st = ADASAP_OK;
#define ENS(buf, bytes) \
  if ((st = h->buf.ensure((size_t)(bytes))) != ADASAP_OK) return fail(st)
  ENS(V, n * k * ss);
  ENS(Z, n * k * ss);
  const bool ard = cfg->n_lengthscale == d && d > 1;
  if (ard) {
    ENS(Xs, (size_t)n * d * 8);
    ENS(iell, (size_t)d * 8);
  }
  ENS(Bdev, b * 8);
  ENS(Bslot[0], b * 8);
  ENS(Bslot[1], b * 8);
  ENS(XB, b * d * (ard ? 8 : dt_size(h->dtype)));
  ENS(G, b * k * 8);
  ENS(D, b * k * 8);
  ENS(Om, b * r * 8);
  ENS(Ysk, b * r * 8);
  ENS(Bm, b * r * 8);
  ENS(U, b * r * 8);
  ENS(Mo, r * r * 8);
  ENS(Qo, r * r * 8);
  ENS(Rinv, r * r * 8);
  ENS(H, r * r * 8);
  ENS(Vr, r * r * 8);
  ENS(T, r * r * 8);
  ENS(evals, r * 8);
  ENS(S, r * 8);
  ENS(cinv, r * 8);
  ENS(cisq, r * 8);
  ENS(coef, (size_t)r * (k > 1 ? k : 1) * 8);
  ENS(coef2, (size_t)r * 8);
  ENS(rot, jacobi_rot_capacity(r) * 8);
  ENS(vv, b * 8);
  ENS(ww, b * 8);
  ENS(uu, b * 8);
  ENS(zz, b * 8);
  ENS(scb, sizeof(IterScalars));
  if (cfg->precond == ADASAP_PRECOND_EXACT) {
    ENS(Hx, (size_t)b * b * 8);
    ENS(Linv, exact_linv_doubles(b) * 8);
  }
#undef ENS
  if (hipHostMalloc((void**)&h->Bhost[0], b * sizeof(int64_t)) != hipSuccess ||
      hipHostMalloc((void**)&h->Bhost[1], b * sizeof(int64_t)) != hipSuccess) {
    set_error("pinned host allocation failed");
    return fail(ADASAP_ERR_OOM);
  }
  if (hipEventCreateWithFlags(&h->bev[0], hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&h->bev[1], hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&h->ev_fork, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&h->ev_join, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&h->ev_sketch, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&h->ev_bup, hipEventDisableTiming) != hipSuccess ||
      hipStreamCreateWithFlags(&h->s2, hipStreamNonBlocking) != hipSuccess) {
    set_error("event creation failed");
    return fail(ADASAP_ERR_DEVICE);
  }
  if (hipMemsetAsync(h->scb.p, 0, sizeof(IterScalars), h->s) != hipSuccess) return fail(ADASAP_ERR_DEVICE);
  if (ard) {
    // per-coordinate lengthscales: every kernel value is computed from x_j / ell_j at ell = 1
    h->inv_ell.resize(d);
    for (int j = 0; j < d; ++j) h->inv_ell[j] = 1.0 / cfg->lengthscales[j];
    h->cfg.lengthscales = nullptr;  // the caller's array is not kept
    if (hipMemcpyAsync(h->iell.p, h->inv_ell.data(), (size_t)d * 8, hipMemcpyHostToDevice, h->s) !=
        hipSuccess)
      return fail(ADASAP_ERR_DEVICE);
    if ((st = scale_columns(n, d, X, h->dtype, h->iell.as<double>(), h->Xs.as<double>(), h->s)) !=
        ADASAP_OK)
      return fail(st);
    h->Xk = h->Xs.p;
    h->xkt = DT::F64;
    h->ellk = 1.0;
  }
  if (h->use_mfma) {
    // the Step-I product runs as one resident round on 7/8 of the workgroup slots, so that
    // the second stream's sketch, Nystrom and powering kernels find room
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cus > 0)
      h->mw.cap_cus = cus;
    st = mfma_pack_create(h->pack, n, d, k, h->Xk, h->xkt, cfg->kernel, h->ellk, h->s);
    if (st == ADASAP_ERR_UNSUPPORTED && cfg->precision == ADASAP_FP32) {
      h->use_mfma = false;  // coordinates outside the float16 range: vector-ALU products
    } else if (st != ADASAP_OK) {
      return fail(st);
    }
    h->fused = h->use_mfma && cfg->precision == ADASAP_MIXED && cfg->accel && cfg->grad_at_z;
  }
  if (hipStreamSynchronize(h->s) != hipSuccess) return fail(ADASAP_ERR_DEVICE);
  *out = h;
  return ADASAP_OK;
}

adasap_status_t adasap_solve(adasap_handle_t h, void* W, adasap_report_t* report) {
  if (!h) return invalid("handle is null");
  if (!W) return invalid("W must be a non-null device pointer");
  const adasap_config_t& c = h->cfg;
  const int64_t nk = h->n * h->k;
  adasap_report_t rep;
  std::memset(&rep, 0, sizeof(rep));
  rep.relres = -1;
  rep.relres_maxcol = -1;
  h->t_done = -1;
  int nf = 0;
  ADASAP_TRY(any_nonfinite(h->n * h->d, h->X, h->dtype, &nf, h->tmp, h->s));
  if (!nf) ADASAP_TRY(any_nonfinite(nk, h->Y, h->dtype, &nf, h->tmp, h->s));
  if (!nf) ADASAP_TRY(any_nonfinite(nk, W, h->dtype, &nf, h->tmp, h->s));
  if (nf) {
    set_error("X, Y or W0 contains NaN or Inf");
    return ADASAP_ERR_NONFINITE;
  }
  ADASAP_TRY(ensure_trace(h, c.max_iters * (1 + c.refine_sweeps)));
  // V_0 = Z_0 = W_0
  ADASAP_TRY(convert(nk, W, h->dtype, h->V.p, h->st, h->s));
  ADASAP_TRY(convert(nk, W, h->dtype, h->Z.p, h->st, h->s));
  int64_t trace_pos = 0;
  h->kev_used = 0;
  h->step1_ms = 0;
  double relres = -1, relmax = -1;
  ADASAP_TRY(run_sweep(h, 0, h->Y, h->dtype, W, 0, c.max_iters, rep.iters, relres, relmax,
                       rep.solve_ms, rep.check_ms, trace_pos));
  // float64 iterative refinement: R = Y - (K + lambda I) W, solve for the correction, add it
  for (int sw = 1; sw <= c.refine_sweeps; ++sw) {
    ADASAP_TRY(h->rhs.ensure((size_t)nk * sizeof(double)));
    ADASAP_TRY(h->delta_w.ensure((size_t)nk * dt_size(h->dtype)));
    double rr = 0;
    ADASAP_TRY(residual_h(h, W, h->dtype, h->Y, h->dtype, &rr, nullptr, false));
    // rhs = -(K W + lambda W - Y)
    ADASAP_TRY(scale_store(nk, h->res.as<double>(), -1.0, h->rhs.p, DT::F64, h->s));
    ADASAP_HIP(hipMemsetAsync(h->delta_w.p, 0, (size_t)nk * dt_size(h->dtype), h->s));
    ADASAP_HIP(hipMemsetAsync(h->V.p, 0, (size_t)nk * dt_size(h->st), h->s));
    ADASAP_HIP(hipMemsetAsync(h->Z.p, 0, (size_t)nk * dt_size(h->st), h->s));
    double r2 = -1, m2 = -1;
    ADASAP_TRY(run_sweep(h, PURPOSE_SWEEP_STRIDE * (uint64_t)sw, h->rhs.p, DT::F64, h->delta_w.p,
                         0, c.max_iters, rep.iters, r2, m2, rep.solve_ms, rep.check_ms, trace_pos));
    ADASAP_TRY(add_inplace(nk, W, h->dtype, h->delta_w.p, h->dtype, h->s));
    rep.refine_done = sw;
    relres = -1;
  }
  if (c.refine_sweeps > 0 && c.tol > 0) {
    auto c0 = std::chrono::steady_clock::now();
    ADASAP_TRY(residual_h(h, W, h->dtype, h->Y, h->dtype, &relres, &relmax, false));
    rep.check_ms += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - c0).count();
  }
  ADASAP_TRY(finish_report(h, rep, trace_pos, relres, relmax));
  if (c.refine_sweeps == 0 && !c.tail_average) h->t_done = rep.iters;
  if (report) *report = rep;
  return rep.status == ADASAP_OK ? ADASAP_OK : (adasap_status_t)rep.status;
}

adasap_status_t adasap_solve_more(adasap_handle_t h, void* W, int64_t iters,
                                  adasap_report_t* report) {
  if (!h) return invalid("handle is null");
  if (!W) return invalid("W must be a non-null device pointer");
  if (iters < 1) return invalid("iters must be >= 1");
  if (h->t_done < 0)
    return invalid("no solve to continue (none run yet, or it used refinement sweeps or tail "
                   "averaging, or failed)");
  adasap_report_t rep;
  std::memset(&rep, 0, sizeof(rep));
  rep.relres = -1;
  rep.relres_maxcol = -1;
  const int64_t t0 = h->t_done;
  h->t_done = -1;
  ADASAP_TRY(ensure_trace(h, iters));
  int64_t trace_pos = 0;
  h->kev_used = 0;
  h->step1_ms = 0;
  double relres = -1, relmax = -1;
  ADASAP_TRY(run_sweep(h, 0, h->Y, h->dtype, W, t0, iters, rep.iters, relres, relmax, rep.solve_ms,
                       rep.check_ms, trace_pos));
  ADASAP_TRY(finish_report(h, rep, trace_pos, relres, relmax));
  h->t_done = t0 + rep.iters;
  if (report) *report = rep;
  return rep.status == ADASAP_OK ? ADASAP_OK : (adasap_status_t)rep.status;
}

adasap_status_t adasap_predict(adasap_handle_t h, const void* W, int64_t m, const void* Xstar,
                               void* out) {
  if (!h) return invalid("handle is null");
  if (m < 0) return invalid("m must be >= 0");
  if (m == 0) return ADASAP_OK;
  if (!W || !Xstar || !out) return invalid("W, Xstar and out must be non-null device pointers");
  ADASAP_TRY(predict_h(h, W, m, Xstar, out));
  ADASAP_HIP(hipStreamSynchronize(h->s));
  return ADASAP_OK;
}

adasap_status_t adasap_posterior_samples(adasap_handle_t h, const void* W, int64_t m,
                                         const void* Xstar, const void* prior_star, void* out) {
  if (!h) return invalid("handle is null");
  if (m < 0) return invalid("m must be >= 0");
  if (m == 0) return ADASAP_OK;
  if (!W || !Xstar || !out) return invalid("W, Xstar and out must be non-null device pointers");
  if (h->k > 1 && !prior_star) return invalid("prior_star must be a device array of m x (k - 1)");
  ADASAP_TRY(predict_h(h, W, m, Xstar, out));
  ADASAP_TRY(pathwise_combine(m, h->k, prior_star, h->dtype, out, h->dtype, h->s));
  ADASAP_HIP(hipStreamSynchronize(h->s));
  return ADASAP_OK;
}

adasap_status_t adasap_residual(adasap_handle_t h, const void* W, double* relres,
                                double* relres_maxcol) {
  if (!h) return invalid("handle is null");
  if (!W) return invalid("W must be a non-null device pointer");
  return residual_h(h, W, h->dtype, h->Y, h->dtype, relres, relres_maxcol, false);
}

adasap_status_t adasap_residual_rows(adasap_handle_t h, const void* W, int64_t m, uint64_t seed,
                                     double* relres, double* relres_maxcol, int64_t* rows_out) {
  if (!h) return invalid("handle is null");
  return residual_rows_h(h, W, h->dtype, h->Y, h->dtype, m, seed, false, relres, relres_maxcol,
                         nullptr, rows_out);
}

adasap_status_t adasap_residual_rows_f64(adasap_handle_t h, const void* W, int64_t m,
                                         uint64_t seed, double* relres, double* relres_maxcol,
                                         double* rel_se, int64_t* rows_out) {
  if (!h) return invalid("handle is null");
  return residual_rows_h(h, W, h->dtype, h->Y, h->dtype, m, seed, true, relres, relres_maxcol,
                         rel_se, rows_out);
}

adasap_status_t adasap_block_gradient(adasap_handle_t h, int64_t t, const void* Z, int64_t* B_out,
                                      double* G_out) {
  if (!h) return invalid("handle is null");
  if (t < 0) return invalid("t must be >= 0");
  if (!Z || !G_out) return invalid("Z and G_out must be non-null device pointers");
  const int64_t b = h->cfg.block_size;
  ADASAP_HIP(hipEventSynchronize(h->bev[0]));
  sample_block_host(h->cfg.seed, PURPOSE_B, (uint64_t)t, h->n, b, h->Bhost[0]);
  ADASAP_HIP(hipMemcpyAsync(h->Bdev.p, h->Bhost[0], b * sizeof(int64_t), hipMemcpyHostToDevice, h->s));
  ADASAP_HIP(hipEventRecord(h->bev[0], h->s));
  const int64_t* B = h->Bdev.as<int64_t>();
  ADASAP_TRY(block_gradient_h(h, B, Z, h->dtype, h->Y, h->dtype, G_out, h->s));
  if (B_out)
    ADASAP_HIP(hipMemcpyAsync(B_out, B, b * sizeof(int64_t), hipMemcpyDeviceToDevice, h->s));
  ADASAP_HIP(hipStreamSynchronize(h->s));
  return ADASAP_OK;
}

adasap_status_t adasap_get_trace(adasap_handle_t h, double* eta, double* rho, double* lambda_hat,
                                 int64_t count) {
  if (!h) return invalid("handle is null");
  if (count < 0) return invalid("count must be >= 0");
  const int64_t m = count < (int64_t)h->eta_tr.size() ? count : (int64_t)h->eta_tr.size();
  for (int64_t i = 0; i < m; ++i) {
    if (eta) eta[i] = h->eta_tr[i];
    if (rho) rho[i] = h->rho_tr[i];
    if (lambda_hat) lambda_hat[i] = h->lh_tr[i];
  }
  return ADASAP_OK;
}

void adasap_destroy(adasap_handle_t h) {
  if (!h) return;
  if (h->s) (void)hipStreamSynchronize(h->s);
  delete h;
}

adasap_status_t adasap_sample_block(uint64_t seed, uint64_t purpose, uint64_t t, int64_t n,
                                    int64_t b, int64_t* out) {
  if (!out) return invalid("out is null");
  if (n < 1 || b < 1 || b > n) return invalid("need 1 <= b <= n");
  sample_block_host(seed, purpose, t, n, b, out);
  return ADASAP_OK;
}

adasap_status_t adasap_normals(uint64_t seed, uint64_t purpose, uint64_t t, int64_t count,
                               double* out, void* stream) {
  if (count < 0) return invalid("count must be >= 0");
  if (count > 0 && !out) return invalid("out is null");
  ADASAP_TRY(normals_dev(seed, purpose, t, count, out, static_cast<hipStream_t>(stream)));
  ADASAP_HIP(hipStreamSynchronize(static_cast<hipStream_t>(stream)));
  return ADASAP_OK;
}

adasap_status_t adasap_kblock_matmul(int32_t kernel, double lengthscale, int32_t precision,
                                     int64_t m, int64_t n, int32_t d, int32_t k, const void* Xr,
                                     const void* Xc, const void* R, void* out, int32_t dtype,
                                     void* stream) {
  if (kernel < 0 || kernel > 3) return invalid("unknown kernel");
  if (!finite_pos(lengthscale)) return invalid("lengthscale must be finite and > 0");
  if (precision < 0 || precision > 2) return invalid("unknown precision");
  if (m < 0 || n < 0) return invalid("m and n must be >= 0");
  if (d < 1 || d > 64) return invalid("d must be in [1, 64]");
  if (k < 1 || k > 128) return invalid("k must be in [1, 128]");
  if (precision == ADASAP_MIXED && d > 16) return invalid("MIXED precision needs d <= 16");
  if (dtype != ADASAP_DTYPE_F32 && dtype != ADASAP_DTYPE_F64) return invalid("unknown dtype");
  if (m == 0) return ADASAP_OK;
  if (!Xr || !out || (n > 0 && (!Xc || !R))) return invalid("null device pointer");
  hipStream_t s = static_cast<hipStream_t>(stream);
  DevBuf part;
  KbEpilogue none;
  const DT t = to_dt(dtype);
  if (precision == ADASAP_MIXED && n > 0) {
    MfmaPack pk;
    MfmaWork w;
    DevBuf rowq;
    ADASAP_TRY(mfma_pack_create(pk, n, d, k, Xc, t, kernel, lengthscale, s));
    ADASAP_TRY(mfma_points(pk, Xr, t, m, rowq, s));
    ADASAP_TRY(mfma_product_rows(pk, rowq.p, m, R, t, k, mfma_mode_f16(), out, t, w, s));
    ADASAP_HIP(hipStreamSynchronize(s));
    return ADASAP_OK;
  }
  ADASAP_TRY(kblock_valu(kernel, lengthscale, precision == ADASAP_FP64 ? ADASAP_FP64 : ADASAP_FP32,
                         m, n, d, k, Xr, nullptr, t, Xc, R, t, k, out, t, k, none, part, s));
  ADASAP_HIP(hipStreamSynchronize(s));
  return ADASAP_OK;
}

adasap_status_t adasap_nystrom(int64_t b, int32_t r, const double* Ysk, const double* Omega,
                               double eps, double* U, double* S, double* delta, void* stream) {
  if (b < 1 || r < 1 || r > 128 || r > b) return invalid("need 1 <= r <= min(b, 128)");
  if (!Ysk || !Omega || !U || !S) return invalid("null device pointer");
  if (!(eps >= 0) || !std::isfinite(eps)) return invalid("eps must be finite and >= 0");
  hipStream_t s = static_cast<hipStream_t>(stream);
  DevBuf Mo, Qo, Rinv, Bm, H, ev, Vr, T, ci, cq, rot, scb, part;
  ADASAP_TRY(Mo.ensure(r * r * 8));
  ADASAP_TRY(Qo.ensure(r * r * 8));
  ADASAP_TRY(Rinv.ensure(r * r * 8));
  ADASAP_TRY(Bm.ensure(b * r * 8));
  ADASAP_TRY(H.ensure(r * r * 8));
  ADASAP_TRY(ev.ensure(r * 8));
  ADASAP_TRY(Vr.ensure(r * r * 8));
  ADASAP_TRY(T.ensure(r * r * 8));
  ADASAP_TRY(ci.ensure(r * 8));
  ADASAP_TRY(cq.ensure(r * 8));
  ADASAP_TRY(rot.ensure(jacobi_rot_capacity(r) * 8));
  ADASAP_TRY(scb.ensure(sizeof(IterScalars)));
  ADASAP_HIP(hipMemsetAsync(scb.p, 0, sizeof(IterScalars), s));
  IterScalars* sc = scb.as<IterScalars>();
  ADASAP_TRY(gram(b, r, r, Omega, DT::F64, r, Ysk, DT::F64, r, Mo.as<double>(), nullptr, part, s));
  ADASAP_TRY(gram(b, r, r, Omega, DT::F64, r, Omega, DT::F64, r, Qo.as<double>(), nullptr, part, s));
  ADASAP_TRY(nys_core(r, Mo.as<double>(), Qo.as<double>(), eps, Rinv.as<double>(), nullptr, sc, s));
  ADASAP_TRY(gemm_rm(b, r, r, Ysk, Omega, &sc->delta, r, Rinv.as<double>(), Bm.as<double>(), r,
                     nullptr, 0, nullptr, 0, s));
  ADASAP_TRY(gram(b, r, r, Bm.p, DT::F64, r, Bm.p, DT::F64, r, H.as<double>(), nullptr, part, s));
  ADASAP_TRY(jacobi_eig(r, H.as<double>(), ev.as<double>(), Vr.as<double>(), rot.as<double>(), sc, s));
  ADASAP_TRY(nys_finalize(r, ev.as<double>(), Vr.as<double>(), 1, 0.0, 1.0, S, T.as<double>(),
                          ci.as<double>(), cq.as<double>(), sc, s));
  ADASAP_TRY(gemm_rm(b, r, r, Bm.as<double>(), nullptr, nullptr, r, T.as<double>(), U, r, nullptr,
                     0, nullptr, 0, s));
  IterScalars hs;
  ADASAP_HIP(hipMemcpyAsync(&hs, sc, sizeof(hs), hipMemcpyDeviceToHost, s));
  ADASAP_HIP(hipStreamSynchronize(s));
  if (delta) ADASAP_HIP(hipMemcpy(delta, &hs.delta, sizeof(double), hipMemcpyHostToDevice));
  if (hs.failed) {
    set_error("Nystrom core not positive definite after shift retries");
    return ADASAP_ERR_NOT_PD;
  }
  return ADASAP_OK;
}

adasap_status_t adasap_precond_apply(int64_t b, int32_t r, int32_t k, const double* U,
                                     const double* S, double rho, int32_t power, const double* G,
                                     double* out, void* stream) {
  if (b < 1 || r < 1 || r > 128 || r > b || k < 1 || k > 128) return invalid("bad sizes");
  if (!finite_pos(rho)) return invalid("rho must be finite and > 0");
  if (power != 0 && power != 1) return invalid("power must be 0 or 1");
  if (!U || !S || !G || !out) return invalid("null device pointer");
  hipStream_t s = static_cast<hipStream_t>(stream);
  DevBuf coefs, coef, scb, part;
  ADASAP_TRY(coefs.ensure(r * 8));
  ADASAP_TRY(coef.ensure((size_t)r * k * 8));
  ADASAP_TRY(scb.ensure(sizeof(IterScalars)));
  ADASAP_TRY(woodbury_coefs(r, S, rho, power, coefs.as<double>(), scb.as<IterScalars>(), s));
  IterScalars* sc = scb.as<IterScalars>();
  ADASAP_TRY(gram(b, r, k, U, DT::F64, r, G, DT::F64, k, coef.as<double>(), coefs.as<double>(), part, s));
  ADASAP_TRY(gemm_rm(b, r, k, U, nullptr, nullptr, r, coef.as<double>(), out, k, G, k, &sc->rho,
                     power == 0 ? 1 : 2, s));
  ADASAP_HIP(hipStreamSynchronize(s));
  return ADASAP_OK;
}

const char* adasap_last_error(void) { return g_last_error.c_str(); }

const char* adasap_status_string(adasap_status_t s) {
  switch (s) {
    case ADASAP_OK: return "ok";
    case ADASAP_ERR_INVALID_ARG: return "invalid argument";
    case ADASAP_ERR_OOM: return "out of memory";
    case ADASAP_ERR_DEVICE: return "device error";
    case ADASAP_ERR_NOT_PD: return "Nystrom core not positive definite";
    case ADASAP_ERR_NONFINITE: return "non-finite values";
    case ADASAP_ERR_UNSUPPORTED: return "unsupported";
    case ADASAP_ERR_NOT_CONVERGED: return "not converged";
    default: return "unknown status";
  }
}

}  // extern "C"
