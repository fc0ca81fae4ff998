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
                                  hipStream_t s);

}  // namespace adasap
