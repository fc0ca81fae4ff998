// Batched ADASAP: many independent GP problems of uneven size solved together, every
// iteration advancing all of them with one launch per step (Alg. 2 for each problem).
//
// Shapes that are equal across the batch (block size b, rank r, one right-hand side) make
// every block-level array a [P][...] stack, so the sketch, the Nystrom factorisation, the
// powering and the Woodbury/Nesterov steps run as single batched launches (grid dimension =
// problem).  The step-I products K(X_B, X) Z, whose column counts differ per problem, run in
// one persistent launch that drains a work queue of (problem, row workgroup, tile chunk)
// items; partial sums are added per problem in a fixed order, so results are deterministic.
//
// Layout: the points of problem p occupy rows row_off[p] .. row_off[p] + 32*ntiles[p] of a
// global padded row space (padding rows stay zero); V, Z, W and Y live on those rows in
// float32; block indices are global rows.  Problem p draws its random numbers with seed + p.
#include <chrono>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "internal.h"
#include "mfma.h"

namespace adasap {

adasap_status_t colsq(int64_t rows, int k, const void* a, DT t, int64_t lda, double* out,
                      DevBuf& tmp, hipStream_t s);
adasap_status_t mfma_batch_residual(const MfmaBatchPack& bp, int p, const void* W, DT wt,
                                    const void* Y, DT yt, double lam, double* res, MfmaWork& w,
                                    hipStream_t s);

namespace {

// copy problem p's n x 1 user array into (dir 0) or out of (dir 1) the padded global rows
__global__ void scatter_rows_kernel(int64_t n, const void* __restrict__ src, DT st,
                                    float* __restrict__ dst_pad) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n)
    dst_pad[i] = st == DT::F64 ? (float)static_cast<const double*>(src)[i] : static_cast<const float*>(src)[i];
}

__global__ void gather_rows_out_kernel(int64_t n, const float* __restrict__ src_pad,
                                       void* __restrict__ dst, DT dt) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (dt == DT::F64) static_cast<double*>(dst)[i] = (double)src_pad[i];
  else static_cast<float*>(dst)[i] = src_pad[i];
}

__global__ void fill_row_prob_kernel(int64_t rows, int32_t* __restrict__ row_prob, int p,
                                     int64_t off) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < rows) row_prob[off + i] = p;
}

// step-I tile shapes chosen by the autotuner, kept for the life of the process per device and
// batch shape (kernel, block size, and every problem's column-tile count and dimension)
struct TuneKey {
  int dev, kern;
  int64_t b;
  uint64_t shape;
  bool operator<(const TuneKey& o) const {
    if (dev != o.dev) return dev < o.dev;
    if (kern != o.kern) return kern < o.kern;
    if (b != o.b) return b < o.b;
    return shape < o.shape;
  }
};
struct TuneVal {
  int rt, wg_per_cu, chunk;
};
std::mutex tune_mu;
std::map<TuneKey, TuneVal> tune_cache;

TuneKey tune_key(int dev, const MfmaBatchPack& bp, int64_t b) {
  uint64_t h = 1469598103934665603ull;  // FNV-1a over (problems, tiles, d) of every problem
  auto mix = [&](uint64_t v) {
    for (int i = 0; i < 8; ++i) {
      h ^= (v >> (8 * i)) & 0xff;
      h *= 1099511628211ull;
    }
  };
  mix((uint64_t)bp.P);
  for (int p = 0; p < bp.P; ++p) {
    mix((uint64_t)bp.ntiles[p]);
    mix((uint64_t)bp.d[p]);
  }
  return TuneKey{dev, bp.kern, b, h};
}

bool tune_lookup(const TuneKey& k, TuneVal& v) {
  std::lock_guard<std::mutex> g(tune_mu);
  auto it = tune_cache.find(k);
  if (it == tune_cache.end()) return false;
  v = it->second;
  return true;
}

void tune_store(const TuneKey& k, const TuneVal& v) {
  std::lock_guard<std::mutex> g(tune_mu);
  tune_cache[k] = v;
}

adasap_status_t invalid(const std::string& m) {
  set_error(m);
  return ADASAP_ERR_INVALID_ARG;
}

}  // namespace
}  // namespace adasap

using namespace adasap;

extern "C" adasap_status_t adasap_solve_batch(const adasap_problem_t* probs, int32_t count,
                                              const adasap_config_t* cfg, int32_t dtype,
                                              void* stream, adasap_report_t* reports) {
  if (!probs || count < 1) return invalid("need at least one problem");
  if (!cfg || cfg->struct_size != sizeof(adasap_config_t)) return invalid("config is null or has the wrong size");
  if (dtype != ADASAP_DTYPE_F32 && dtype != ADASAP_DTYPE_F64) return invalid("unknown dtype");
  if (cfg->kernel < 0 || cfg->kernel > 3) return invalid("unknown kernel");
  if (!(cfg->lambda > 0) || !std::isfinite(cfg->lambda)) return invalid("lambda must be finite and > 0");
  if (cfg->precond != ADASAP_PRECOND_NYSTROM) return invalid("batched solves use the Nystrom preconditioner");
  if (cfg->precision != ADASAP_FP32) return invalid("batched solves run in FP32 precision");
  if (!cfg->accel || !cfg->grad_at_z || cfg->tail_average) return invalid("batched solves use the accelerated step with the gradient at Z");
  if (cfg->power_iters < 1 || cfg->power_iters > 1000) return invalid("power_iters must be in [1, 1000]");
  if (cfg->max_iters < 0) return invalid("max_iters must be >= 0");
  if (cfg->rho_rule != 0 && cfg->rho_rule != 1) return invalid("rho_rule must be 0 or 1");
  if (cfg->rho_rule == 1 && !(cfg->rho > 0)) return invalid("rho must be > 0");
  if (cfg->n_lengthscale > 1 || cfg->outputscale != 1.0)
    return invalid("batched solves take one scalar lengthscale per problem and unit output scale");
  const int P = count;
  const int64_t b = cfg->block_size;
  const int r = cfg->rank;
  if (b < 1) return invalid("block size must be >= 1");
  if (r < 1 || r > 128 || r > b) return invalid("rank must be in [1, min(b, 128)]");
  std::vector<int64_t> n(P);
  std::vector<int> d(P);
  std::vector<double> ell(P), coefs(3 * (size_t)P);
  std::vector<const void*> Xp(P);
  const double mu = cfg->mu > 0 ? cfg->mu : cfg->lambda;
  for (int p = 0; p < P; ++p) {
    const adasap_problem_t& q = probs[p];
    if (q.k != 1) return invalid("batched solves take one right-hand side per problem");
    if (q.d < 1 || q.d > 16) return invalid("batched solves need 1 <= d <= 16");
    if (q.n < b) return invalid("every problem needs n >= block size");
    if (!q.X || !q.Y || !q.W) return invalid("null device pointer in a problem");
    if (!(q.lengthscale > 0) || !std::isfinite(q.lengthscale)) return invalid("lengthscale must be > 0");
    n[p] = q.n;
    d[p] = q.d;
    ell[p] = q.lengthscale;
    Xp[p] = q.X;
    const double nu = cfg->nu > 0 ? cfg->nu : (double)q.n / (double)b;
    if (mu > nu) return invalid("need mu <= nu for every problem");
    coefs[3 * p] = 1.0 - std::sqrt(mu / nu);
    coefs[3 * p + 1] = 1.0 / std::sqrt(mu * nu);
    coefs[3 * p + 2] = 1.0 / (1.0 + coefs[3 * p + 1] * nu);
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  const DT dt = dtype == ADASAP_DTYPE_F64 ? DT::F64 : DT::F32;
  const double lam = cfg->lambda;

  MfmaBatchPack bp;
  ADASAP_TRY(mfma_batch_pack_create(bp, P, n.data(), d.data(), Xp.data(), dt, ell.data(),
                                    cfg->kernel, s));
  MfmaQueue q;
  ADASAP_TRY(mfma_batch_queue_create(bp, b, 64, 4, q, s));
  const int64_t R = bp.rows_total;
  DevBuf V, Z, Wp, Yp, rowp, dcoef, Bdev, G, D, Om, Ysk, Mo, Qo, Rinv, Bm, H, ev, Vr, T, S, cinv,
      cisq, U, rot, vv, ww, uu, zz, coef, coef2, scb, colsB, pg, pg2, pd, res, colq, tmp;
  MfmaWork w1, w2;
  const size_t Pb = (size_t)P * b, Pbr = Pb * r, Prr = (size_t)P * r * r;
  ADASAP_TRY(V.ensure(R * 4));
  ADASAP_TRY(Z.ensure(R * 4));
  ADASAP_TRY(Wp.ensure(R * 4));
  ADASAP_TRY(Yp.ensure(R * 4));
  ADASAP_TRY(rowp.ensure(R * 4));
  ADASAP_TRY(dcoef.ensure(coefs.size() * 8));
  ADASAP_TRY(Bdev.ensure((Pb + 1) * 8));
  ADASAP_TRY(G.ensure(Pb * 8));
  ADASAP_TRY(D.ensure(Pb * 8));
  ADASAP_TRY(Om.ensure(Pbr * 8));
  ADASAP_TRY(Ysk.ensure(Pbr * 8));
  ADASAP_TRY(Bm.ensure(Pbr * 8));
  ADASAP_TRY(U.ensure(Pbr * 8));
  ADASAP_TRY(Mo.ensure(Prr * 8));
  ADASAP_TRY(Qo.ensure(Prr * 8));
  ADASAP_TRY(Rinv.ensure(Prr * 8));
  ADASAP_TRY(H.ensure(Prr * 8));
  ADASAP_TRY(Vr.ensure(Prr * 8));
  ADASAP_TRY(T.ensure(Prr * 8));
  ADASAP_TRY(ev.ensure((size_t)P * r * 8));
  ADASAP_TRY(S.ensure((size_t)P * r * 8));
  ADASAP_TRY(cinv.ensure((size_t)P * r * 8));
  ADASAP_TRY(cisq.ensure((size_t)P * r * 8));
  ADASAP_TRY(coef.ensure((size_t)P * r * 8));
  ADASAP_TRY(coef2.ensure((size_t)P * r * 8));
  ADASAP_TRY(rot.ensure((size_t)P * jacobi_rot_capacity(r) * 8));
  ADASAP_TRY(vv.ensure(Pb * 8));
  ADASAP_TRY(ww.ensure(Pb * 8));
  ADASAP_TRY(uu.ensure(Pb * 8));
  ADASAP_TRY(zz.ensure(Pb * 8));
  ADASAP_TRY(scb.ensure((size_t)P * sizeof(IterScalars)));
  ADASAP_HIP(hipMemsetAsync(V.p, 0, R * 4, s));
  ADASAP_HIP(hipMemsetAsync(Z.p, 0, R * 4, s));
  ADASAP_HIP(hipMemsetAsync(Wp.p, 0, R * 4, s));
  ADASAP_HIP(hipMemsetAsync(Yp.p, 0, R * 4, s));
  ADASAP_HIP(hipMemsetAsync(scb.p, 0, (size_t)P * sizeof(IterScalars), s));
  ADASAP_HIP(hipMemcpyAsync(dcoef.p, coefs.data(), coefs.size() * 8, hipMemcpyHostToDevice, s));
  for (int p = 0; p < P; ++p) {
    const unsigned g = (unsigned)((n[p] + 255) / 256);
    float* yp = Yp.as<float>() + bp.row_off[p];
    hipLaunchKernelGGL(scatter_rows_kernel, dim3(g), dim3(256), 0, s, n[p], probs[p].Y, dt, yp);
    // W_0 from the caller (zeros = cold start); V_0 = Z_0 = W_0
    hipLaunchKernelGGL(scatter_rows_kernel, dim3(g), dim3(256), 0, s, n[p], (const void*)probs[p].W,
                       dt, Z.as<float>() + bp.row_off[p]);
    hipLaunchKernelGGL(scatter_rows_kernel, dim3(g), dim3(256), 0, s, n[p], (const void*)probs[p].W,
                       dt, V.as<float>() + bp.row_off[p]);
    const int64_t rows = bp.ntiles[p] * 32;
    hipLaunchKernelGGL(fill_row_prob_kernel, dim3((unsigned)((rows + 255) / 256)), dim3(256), 0, s,
                       rows, rowp.as<int32_t>(), p, bp.row_off[p]);
    ADASAP_LAUNCH_CHECK();
  }
  hipStream_t s2 = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr, ev_mid = nullptr, k0 = nullptr, k1 = nullptr;
  ADASAP_HIP(hipStreamCreateWithFlags(&s2, hipStreamNonBlocking));
  ADASAP_HIP(hipEventCreateWithFlags(&ev_fork, hipEventDisableTiming));
  ADASAP_HIP(hipEventCreateWithFlags(&ev_join, hipEventDisableTiming));
  ADASAP_HIP(hipEventCreateWithFlags(&ev_mid, hipEventDisableTiming));
  ADASAP_HIP(hipEventCreate(&k0));
  ADASAP_HIP(hipEventCreate(&k1));
  struct Cleanup {
    hipStream_t s2;
    hipEvent_t e[5];
    ~Cleanup() {
      if (s2) (void)hipStreamSynchronize(s2), (void)hipStreamDestroy(s2);
      for (hipEvent_t x : e)
        if (x) (void)hipEventDestroy(x);
    }
  } cleanup{s2, {ev_fork, ev_join, ev_mid, k0, k1}};
  // two pinned upload slots of Pb + 1 entries: every problem's block, then the iteration
  // counter t (read on the device by the random-number kernels, so that a captured round
  // replays with the current t)
  const size_t slot_len = Pb + 1;
  int64_t* Bhost = nullptr;
  if (hipHostMalloc((void**)&Bhost, 2 * slot_len * sizeof(int64_t)) != hipSuccess) {
    set_error("pinned host allocation failed");
    return ADASAP_ERR_OOM;
  }
  struct HostFree {
    int64_t* p;
    ~HostFree() {
      if (p) (void)hipHostFree(p);
    }
  } hf{Bhost};

  IterScalars* sc = scb.as<IterScalars>();
  NestCoef nc{};
  nc.accel = 1;
  nc.z_uses_v_next = cfg->z_uses_v_next ? 1 : 0;
  const double eps = std::ldexp(1.0, -23);
  const unsigned nthreads = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  double solve_ms = 0, step1_ms = 0;
  int step1_timed = 0;
  const int64_t Tmax = cfg->max_iters;
  Batch bBR{P, (int64_t)b * r, (int64_t)b * r, (int64_t)r * r, 0, 0};  // P x b x r Gram operands
  const int64_t* t_dev = Bdev.as<int64_t>() + Pb;
  // events: upload slots, and a ring of per-round timing pairs read back when the ring wraps
  constexpr int RING = 16;
  std::vector<hipEvent_t> slot_ev(2, nullptr), rev(2 * RING, nullptr);
  struct EvFree {
    std::vector<hipEvent_t>* a;
    std::vector<hipEvent_t>* b;
    ~EvFree() {
      for (hipEvent_t e : *a)
        if (e) (void)hipEventDestroy(e);
      for (hipEvent_t e : *b)
        if (e) (void)hipEventDestroy(e);
    }
  } evfree{&slot_ev, &rev};
  for (auto& e : slot_ev) ADASAP_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  for (auto& e : rev) ADASAP_HIP(hipEventCreate(&e));
  auto take_round_time = [&](int64_t u) -> adasap_status_t {
    const int i = (int)(u % RING);
    float ms = 0;
    ADASAP_HIP(hipEventSynchronize(rev[2 * i + 1]));
    ADASAP_HIP(hipEventElapsedTime(&ms, rev[2 * i], rev[2 * i + 1]));
    solve_ms += ms;
    return ADASAP_OK;
  };
  // a captured round (graph) replays every round but the first (eager: it sizes the scratch
  // buffers and runs the autotuner) and the last (eager: it also writes W)
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  bool use_graph = true;
  struct GraphFree {
    hipGraph_t* g;
    hipGraphExec_t* x;
    ~GraphFree() {
      if (*x) (void)hipGraphExecDestroy(*x);
      if (*g) (void)hipGraphDestroy(*g);
    }
  } graphfree{&graph, &graph_exec};
  TuneVal chosen{4, 2, 64};
  int tuned_from_cache = 0;

  // the device work of one round (B_t and t already uploaded); `last` also writes W.  The
  // Gaussian test matrices of round t + 1 are drawn during round t on the main stream, off the
  // chain's critical path, once the sketch products and Grams of round t have read those of
  // round t (from the eigensolvers on, whose one workgroup per problem leaves most of the GPU
  // idle); the first round draws its own.
  auto round = [&](bool last, bool timed, bool first) -> adasap_status_t {
    const int64_t* B = Bdev.as<int64_t>();
    ADASAP_HIP(hipEventRecord(ev_fork, s));
    ADASAP_HIP(hipStreamWaitEvent(s2, ev_fork, 0));
    // step I (main stream): one persistent launch for every problem
    KbEpilogue epg;
    epg.E1 = Z.p;
    epg.e1t = DT::F32;
    epg.e1idx = B;
    epg.lde1 = 1;
    epg.a1 = lam;
    epg.E2 = Yp.p;
    epg.e2t = DT::F32;
    epg.e2idx = B;
    epg.lde2 = 1;
    epg.a2 = -1.0;
    epg.bsIdx = b;
    ADASAP_TRY(mfma_batch_stepI(bp, q, B, b, Z.as<float>(), G.as<double>(), epg, w1, s,
                                timed ? k0 : nullptr, timed ? k1 : nullptr));
    // second stream: sketch, Nystrom factors, step size for every problem
    ADASAP_TRY(mfma_batch_pack_blocks(bp, B, b, colsB, s2));
    if (first) ADASAP_TRY(normals_dev(cfg->seed, PURPOSE_OMEGA, 0, b * r, Om.as<double>(), s2, P, t_dev));
    KbEpilogue none;
    ADASAP_TRY(mfma_batch_block_product(bp, B, b, colsB.p, Om.as<double>(), r, mfma_mode_f16x3(),
                                        Ysk.as<double>(), none, w2, s2));
    ADASAP_TRY(gram(b, r, r, Om.p, DT::F64, r, Ysk.p, DT::F64, r, Mo.as<double>(), nullptr, pg2, s2, bBR));
    ADASAP_TRY(gram(b, r, r, Om.p, DT::F64, r, Om.p, DT::F64, r, Qo.as<double>(), nullptr, pg2, s2, bBR));
    ADASAP_TRY(nys_core(r, Mo.as<double>(), Qo.as<double>(), eps, Rinv.as<double>(), nullptr, sc, s2, P));
    ADASAP_TRY(gemm_rm(b, r, r, Ysk.as<double>(), Om.as<double>(), &sc->delta, r, Rinv.as<double>(),
                       Bm.as<double>(), r, nullptr, 0, nullptr, 0, s2,
                       Batch{P, (int64_t)b * r, (int64_t)r * r, (int64_t)b * r, 0, SC_DOUBLES}));
    ADASAP_TRY(gram(b, r, r, Bm.p, DT::F64, r, Bm.p, DT::F64, r, H.as<double>(), nullptr, pg2, s2, bBR));
    // Om is not read after this point of the round
    ADASAP_HIP(hipEventRecord(ev_mid, s2));
    ADASAP_TRY(jacobi_eig(r, H.as<double>(), ev.as<double>(), Vr.as<double>(), rot.as<double>(), sc, s2, P));
    ADASAP_TRY(nys_finalize(r, ev.as<double>(), Vr.as<double>(), cfg->rho_rule, lam, cfg->rho,
                            S.as<double>(), T.as<double>(), cinv.as<double>(), cisq.as<double>(),
                            sc, s2, P));
    ADASAP_TRY(gemm_rm(b, r, r, Bm.as<double>(), nullptr, nullptr, r, T.as<double>(), U.as<double>(),
                       r, nullptr, 0, nullptr, 0, s2,
                       Batch{P, (int64_t)b * r, (int64_t)r * r, (int64_t)b * r, 0, 0}));
    // P^{-1/2} x (power 1) or P^{-1} x (power 0) for every problem's vector x (P x b)
    auto papply = [&](const double* x, double* out, int power) -> adasap_status_t {
      ADASAP_TRY(gram(b, r, 1, U.p, DT::F64, r, x, DT::F64, 1, coef2.as<double>(),
                      power == 0 ? cinv.as<double>() : cisq.as<double>(), pg2, s2,
                      Batch{P, (int64_t)b * r, (int64_t)b, (int64_t)r, (int64_t)r, 0}));
      return gemm_rm(b, r, 1, U.as<double>(), nullptr, nullptr, r, coef2.as<double>(), out, 1, x, 1,
                     &sc->rho, power == 0 ? 1 : 2, s2,
                     Batch{P, (int64_t)b * r, (int64_t)r, (int64_t)b, (int64_t)b, SC_DOUBLES});
    };
    double* v = vv.as<double>();
    double* wv = ww.as<double>();
    double* u = uu.as<double>();
    double* z = zz.as<double>();
    // powering carried as w = P^{-1/2} v: one P^{-1} apply per step (power_step)
    ADASAP_TRY(normals_dev(cfg->seed, PURPOSE_POW, 0, b, v, s2, P, t_dev));
    ADASAP_TRY(normalize_inplace(b, v, sc, pd, s2, P));
    ADASAP_TRY(papply(v, wv, 1));
    for (int i = 0; i < cfg->power_iters; ++i) {
      KbEpilogue epp;
      epp.E1 = wv;
      epp.e1t = DT::F64;
      epp.lde1 = 1;
      epp.a1 = lam;
      epp.bsE1 = b;
      ADASAP_TRY(mfma_batch_block_product(bp, B, b, colsB.p, wv, 1, mfma_mode_f32v(), u, epp, w2, s2));
      ADASAP_TRY(papply(u, z, 0));
      ADASAP_TRY(power_step(b, wv, u, z, sc, i == cfg->power_iters - 1 ? 1 : 0, s2, P));
    }
    ADASAP_HIP(hipEventRecord(ev_join, s2));
    if (!last) {
      ADASAP_HIP(hipStreamWaitEvent(s, ev_mid, 0));
      ADASAP_TRY(normals_dev(cfg->seed, PURPOSE_OMEGA, 1, b * r, Om.as<double>(), s, P, t_dev));
    }
    ADASAP_HIP(hipStreamWaitEvent(s, ev_join, 0));
    // direction and update (main stream)
    ADASAP_TRY(gram(b, r, 1, U.p, DT::F64, r, G.p, DT::F64, 1, coef.as<double>(), cinv.as<double>(),
                    pg, s, Batch{P, (int64_t)b * r, (int64_t)b, (int64_t)r, (int64_t)r, 0}));
    ADASAP_TRY(gemm_rm(b, r, 1, U.as<double>(), nullptr, nullptr, r, coef.as<double>(), D.as<double>(),
                       1, G.as<double>(), 1, &sc->rho, 1, s,
                       Batch{P, (int64_t)b * r, (int64_t)r, (int64_t)b, (int64_t)b, SC_DOUBLES}));
    ADASAP_TRY(nesterov_dense(R, V.p, Z.p, DT::F32, nc, last ? Wp.p : nullptr, DT::F32, s,
                              rowp.as<int32_t>(), dcoef.as<double>(), 1));
    ADASAP_TRY(nesterov_sparse(b, 1, B, D.as<double>(), V.p, Z.p, DT::F32, nc, sc,
                               last ? Wp.p : nullptr, DT::F32, s, P, dcoef.as<double>()));
    return ADASAP_OK;
  };

  for (int64_t t = 0; t < Tmax; ++t) {
    const int slot = (int)(t & 1);
    int64_t* Bs = Bhost + slot * slot_len;
    // the upload that last read this slot (round t - 2) has completed
    ADASAP_HIP(hipEventSynchronize(slot_ev[slot]));
    // host: every problem's block, drawn in parallel, as global row indices
    {
      std::vector<std::thread> pool;
      for (unsigned th = 0; th < nthreads; ++th)
        pool.emplace_back([&, th]() {
          for (int p = (int)th; p < P; p += (int)nthreads) {
            int64_t* Bp = Bs + (size_t)p * b;
            sample_block_host(cfg->seed + (uint64_t)p, PURPOSE_B, (uint64_t)t, n[p], b, Bp);
            for (int64_t i = 0; i < b; ++i) Bp[i] += bp.row_off[p];
          }
        });
      for (auto& th : pool) th.join();
    }
    Bs[Pb] = t;
    if (t >= RING) ADASAP_TRY(take_round_time(t - RING));
    ADASAP_HIP(hipEventRecord(rev[2 * (t % RING)], s));
    ADASAP_HIP(hipMemcpyAsync(Bdev.p, Bs, slot_len * sizeof(int64_t), hipMemcpyHostToDevice, s));
    ADASAP_HIP(hipEventRecord(slot_ev[slot], s));
    const bool last = t + 1 == Tmax;
    if (t == 0) {
      // autotuner: the step-I launch's tile shape (rows per workgroup), workgroups per CU and
      // work-item size, timed on this batch (second of two launches each) unless the process
      // has tuned the same shapes on this device before
      int dev = 0;
      ADASAP_HIP(hipGetDevice(&dev));
      const TuneKey key = tune_key(dev, bp, b);
      TuneVal tv;
      if (tune_lookup(key, tv)) {
        tuned_from_cache = 1;
      } else {
        float best = 1e30f;
        KbEpilogue none;
        for (int rt : {2, 4})
          for (int wgcu : {2, 4})
            for (int chunk : {16, 32, 64, 128}) {
              MfmaQueue qc;
              qc.wg_per_cu = wgcu;
              ADASAP_TRY(mfma_batch_queue_create(bp, b, chunk, rt, qc, s));
              float ms = 0;
              for (int rep = 0; rep < 2; ++rep) {  // the first launch warms caches and allocations
                ADASAP_TRY(mfma_batch_stepI(bp, qc, Bdev.as<int64_t>(), b, Z.as<float>(),
                                            G.as<double>(), none, w1, s, k0, k1));
                ADASAP_HIP(hipEventSynchronize(k1));
                ADASAP_HIP(hipEventElapsedTime(&ms, k0, k1));
              }
              if (ms < best) {
                best = ms;
                tv = TuneVal{rt, wgcu, chunk};
              }
            }
        tune_store(key, tv);
      }
      chosen = tv;
      q.wg_per_cu = tv.wg_per_cu;
      if (tv.rt != 4 || tv.chunk != 64) ADASAP_TRY(mfma_batch_queue_create(bp, b, tv.chunk, tv.rt, q, s));
    }
    if (t >= 1 && !last && use_graph) {
      if (!graph_exec) {
        // capture this round's device work once; any capture failure leaves the eager rounds
        hipError_t ce = hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed);
        adasap_status_t rst = ce == hipSuccess ? round(false, false, false) : ADASAP_ERR_DEVICE;
        hipGraph_t g = nullptr;
        const hipError_t ee = ce == hipSuccess ? hipStreamEndCapture(s, &g) : ce;
        if (rst == ADASAP_OK && ee == hipSuccess && g &&
            hipGraphInstantiate(&graph_exec, g, nullptr, nullptr, 0) == hipSuccess) {
          graph = g;
        } else {
          if (g) (void)hipGraphDestroy(g);
          graph_exec = nullptr;
          use_graph = false;
          (void)hipGetLastError();
        }
      }
      if (use_graph) ADASAP_HIP(hipGraphLaunch(graph_exec, s));
      else ADASAP_TRY(round(false, false, false));
    } else {
      ADASAP_TRY(round(last, true, t == 0));
      float kms = 0;
      ADASAP_HIP(hipEventSynchronize(k1));
      ADASAP_HIP(hipEventElapsedTime(&kms, k0, k1));
      step1_ms += kms;
      ++step1_timed;
    }
    ADASAP_HIP(hipEventRecord(rev[2 * (t % RING) + 1], s));
  }
  for (int64_t u = Tmax > RING ? Tmax - RING : 0; u < Tmax; ++u) ADASAP_TRY(take_round_time(u));
  // results back to the callers' buffers, per-problem residuals and scalars
  std::vector<IterScalars> hs(P);
  ADASAP_HIP(hipMemcpyAsync(hs.data(), scb.p, (size_t)P * sizeof(IterScalars), hipMemcpyDeviceToHost, s));
  ADASAP_HIP(hipStreamSynchronize(s));
  adasap_status_t status = ADASAP_OK;
  for (int p = 0; p < P; ++p) {
    const unsigned g = (unsigned)((n[p] + 255) / 256);
    if (Tmax > 0)
      hipLaunchKernelGGL(gather_rows_out_kernel, dim3(g), dim3(256), 0, s, n[p],
                         Wp.as<float>() + bp.row_off[p], probs[p].W, dt);
    ADASAP_LAUNCH_CHECK();
    adasap_report_t rep;
    std::memset(&rep, 0, sizeof(rep));
    rep.iters = Tmax;
    rep.solve_ms = solve_ms;
    rep.step1_kernel_ms = step1_ms;
    rep.step1_launches = step1_timed;
    rep.reserved = chosen.chunk;
    rep.tuned_rows_per_wg = 64 * chosen.rt;
    rep.tuned_wg_per_cu = chosen.wg_per_cu;
    rep.tuned_from_cache = tuned_from_cache;
    rep.eta_last = hs[p].eta;
    rep.rho_last = hs[p].rho;
    rep.lambda_hat_last = hs[p].lam_hat;
    rep.delta_last = hs[p].delta;
    rep.relres = -1;
    rep.relres_maxcol = -1;
    if (hs[p].failed) {
      rep.status = ADASAP_ERR_NOT_PD;
      status = ADASAP_ERR_NOT_PD;
    }
    if (cfg->tol > 0 || cfg->check_every > 0) {
      auto c0 = std::chrono::steady_clock::now();
      ADASAP_TRY(res.ensure((size_t)n[p] * 8));
      ADASAP_TRY(colq.ensure(2 * 8));
      ADASAP_TRY(mfma_batch_residual(bp, p, probs[p].W, dt, probs[p].Y, dt, lam, res.as<double>(), w1, s));
      ADASAP_TRY(colsq(n[p], 1, res.p, DT::F64, 1, colq.as<double>(), tmp, s));
      ADASAP_TRY(colsq(n[p], 1, probs[p].Y, dt, 1, colq.as<double>() + 1, tmp, s));
      double hq[2];
      ADASAP_HIP(hipMemcpyAsync(hq, colq.p, 2 * 8, hipMemcpyDeviceToHost, s));
      ADASAP_HIP(hipStreamSynchronize(s));
      rep.relres = hq[1] > 0 ? std::sqrt(hq[0] / hq[1]) : std::sqrt(hq[0]);
      rep.relres_maxcol = rep.relres;
      rep.check_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - c0).count();
    }
    if (reports) reports[p] = rep;
  }
  ADASAP_HIP(hipStreamSynchronize(s));
  if (status != ADASAP_OK) set_error("a Nystrom core was not positive definite after shift retries");
  return status;
}
