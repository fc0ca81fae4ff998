// Matrix-core (MFMA) kernel-block products for gfx950: squared distances from a
// three-term float16 split of the centred, scaled coordinates on v_mfma_f32_16x16x32_f16,
// kernel values on the vector ALUs, and the product with the right-hand side either on the
// matrix cores (float16, or a float16 hi/lo split) or on the vector ALUs (float32, k <= 4).
#pragma once

#include "internal.h"

namespace adasap {

// Packed data of the n points that form the columns (and rows) of every kernel block.
struct MfmaPack {
  int64_t n = 0;
  int d = 0;
  int kern = 0;
  double ell = 1.0;
  int64_t ntiles = 0;   // column tiles of 32 points
  double sigma = 1.0;   // coordinate scale
  DevBuf rowv;          // row vectors, 64 float16 per point (padded to ntiles*32 points)
  DevBuf cols;          // column fragments of all points
  DevBuf centre;        // coordinate mean (float64, d)
  DevBuf flag;
  DevBuf tmp;
};

// Scratch of one caller (packed right-hand side, scales, partial sums).
struct MfmaWork {
  DevBuf rhs, scale, tmp, part;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;  // when set, recorded around the product kernel
  int cap_cus = 0;  // > 0: leave 1/8 of the workgroup slots of this many CUs to a concurrent stream
  hipEvent_t wait_ev = nullptr;  // when set, the product kernel (not the packing) waits for it
};

// A packed right-hand side (see mfma_pack_rhs_full).
struct RhsPacked {
  int mode = 0;
  int nq = 0;
  const void* p = nullptr;
  const float* scale = nullptr;
};

int mfma_mode_f16();    // K and R in float16
int mfma_mode_f16x3();  // K and R split into float16 hi + lo, three products
int mfma_mode_f32v();   // float32 K times float32 R on the vector ALUs (k <= 4)

size_t mfma_pack_bytes(int64_t n, int d, int k);
// centre, scale and pack X (n x d, type xt); fails with UNSUPPORTED if float16 would overflow
adasap_status_t mfma_pack_create(MfmaPack& pk, int64_t n, int d, int k, const void* X, DT xt,
                                 int kern, double ell, hipStream_t s);
// column fragments of the block points B[0..b)
adasap_status_t mfma_pack_block(const MfmaPack& pk, const int64_t* B, int64_t b, DevBuf& colsB,
                                hipStream_t s);
// OUT (m x k, type ot) = K(rows, cols) R + epilogue.  Rows are the pack's points ridx[0..m)
// (or 0..m-1); columns are all n points (colsB == null, R has n rows) or the block points
// packed in colsB (R has ncols rows).  R (type rt, row-major, k columns) is packed here.
// (mfma_product records w.ev0 / w.ev1 around the product kernel when they are set)
adasap_status_t mfma_product(const MfmaPack& pk, const int64_t* ridx, int64_t m,
                             const void* colsB, int64_t ncols, const void* R, DT rt, int k,
                             int mode, void* out, DT ot, const KbEpilogue& ep, MfmaWork& w,
                             hipStream_t s);
// pack an n x k right-hand side once, use it with mfma_product_packed
adasap_status_t mfma_pack_rhs_full(const MfmaPack& pk, const void* R, DT rt, int k, int mode,
                                   MfmaWork& w, RhsPacked& rp, hipStream_t s);
adasap_status_t mfma_product_packed(const MfmaPack& pk, const int64_t* ridx, int64_t m,
                                    const RhsPacked& rp, int k, void* out, DT ot,
                                    const KbEpilogue& ep, MfmaWork& w, hipStream_t s);
// row vectors of query points Xq (m x d) with the pack's centre and scale
adasap_status_t mfma_points(const MfmaPack& pk, const void* Xq, DT xt, int64_t m, DevBuf& rowq,
                            hipStream_t s);
// OUT = K(Xq, X) R for query rows packed by mfma_points
adasap_status_t mfma_product_rows(const MfmaPack& pk, const void* rowq, int64_t m, const void* R,
                                  DT rt, int k, int mode, void* out, DT ot, MfmaWork& w,
                                  hipStream_t s, double kscale = 1.0);

// ---- fused Nesterov update and float16 packing of Z (MIXED path) ------------------------------
// The packed float16 Z of the Step-I product is produced by the update pass itself: fused_init
// packs the starting Z and records column maxima of |V| and |Z|; each fused_update applies the
// Nesterov step (all rows + the rows of B with direction D and sc->eta), writes V, Z (and W
// when non-null) and packs the new Z with scales bounded from the recorded maxima.
struct FusedUpd {
  DevBuf pos;      // int64[n]: (stamp << 32) | j for the rows B[j] of the current block
  DevBuf packed;   // float16 Z in the Step-I operand order
  DevBuf scale;    // float[k] power-of-two column scales of the packed Z
  DevBuf part;     // per-workgroup maxima [nwg][2][k] of |V| and |Z|
  DevBuf dpart;    // per-block column maxima [nblk][k] of |D| (the block's direction)
  int nwg = 0, mode = 0, nq = 0;
  uint32_t stamp = 0;
};
adasap_status_t fused_init(const MfmaPack& pk, FusedUpd& f, int k, const float* V, const float* Z,
                           MfmaWork& w, hipStream_t s);
RhsPacked fused_rhs(const FusedUpd& f);
adasap_status_t fused_update(const MfmaPack& pk, FusedUpd& f, int k, const int64_t* B, int64_t b,
                             const double* D, const IterScalars* sc, const NestCoef& c, float* V,
                             float* Z, void* W, DT wt, hipStream_t s);

// ---- batches of independent problems (all with two K-steps, d <= 16) --------------------------
// Points of problem p occupy rows row_off[p] .. row_off[p] + ntiles[p]*32 of the global row
// space (padding rows are zero); block indices passed to the batch launchers are global rows.
struct MfmaBatchPack {
  int P = 0;
  int kern = 0;
  std::vector<int64_t> n, ntiles, row_off, col_off;
  std::vector<int> d;
  int64_t rows_total = 0;
  DevBuf rowv, cols, centre, flag, dvec, col_off_dev, rhs_off_dev;
};

// Work items (problem, row workgroup, column-tile chunk) of the persistent step-I launch.
struct MfmaQueue {
  int nitems = 0;
  int rows_per_wg = 256;
  int rt = 4;         // row tiles of 16 per wave: 64 rt rows per workgroup (2 or 4)
  int wg_per_cu = 2;  // persistent workgroups per CU (2 or 4)
  int qbeg[9] = {0};  // item ranges of the eight XCDs
  DevBuf items, item_start, nchunk, counter;
};

adasap_status_t mfma_batch_pack_create(MfmaBatchPack& bp, int P, const int64_t* n, const int* d,
                                       const void* const* X, DT xt, const double* ell, int kern,
                                       hipStream_t s);
// column fragments of every problem's block (B: P x b global row indices)
adasap_status_t mfma_batch_pack_blocks(const MfmaBatchPack& bp, const int64_t* B, int64_t b,
                                       DevBuf& colsB, hipStream_t s);
// OUT[p] = K(X_B[p], X_B[p]) R[p] + epilogue for every problem (R, OUT: P x b x k float64)
adasap_status_t mfma_batch_block_product(const MfmaBatchPack& bp, const int64_t* B, int64_t b,
                                         const void* colsB, const double* R, int k, int mode,
                                         double* out, const KbEpilogue& ep, MfmaWork& w,
                                         hipStream_t s);
adasap_status_t mfma_batch_queue_create(const MfmaBatchPack& bp, int64_t b, int64_t chunk_tiles,
                                        int rt, MfmaQueue& q, hipStream_t s);
// G[p] = K(X_B[p], X[p]) Z[p] + epilogue for all problems in one persistent launch
// (Z: float32 on the global padded rows, k = 1)
adasap_status_t mfma_batch_stepI(const MfmaBatchPack& bp, MfmaQueue& q, const int64_t* B, int64_t b,
                                 const float* Z, double* out, const KbEpilogue& ep, MfmaWork& w,
                                 hipStream_t s, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);

}  // namespace adasap
