// Matrix-core (MFMA) kernel-block products for gfx950: squared distances from a
// three-term float16 split of the coordinates on v_mfma_f32_16x16x32_f16, kernel values
// on the vector ALUs, and the product with the right-hand side on the matrix cores.
#pragma once

#include "internal.h"

namespace adasap {

// Packed column data of a point set (the n columns of every kernel block).
struct MfmaPack {
  int64_t n = 0;
  int d = 0;
  int64_t ntiles = 0;   // column tiles of 32
  double shift_scale = 0;
  DevBuf cols;          // packed A-operand fragments of the columns
  DevBuf centre;        // coordinate mean (float64, d) used to centre every point
  DevBuf tmp;
};

size_t mfma_pack_bytes(int64_t n, int d, int k);
adasap_status_t mfma_pack_create(MfmaPack& pk, int64_t n, int d, int k, const void* X, DT xt,
                                 int kern, double ell, hipStream_t s);
size_t mfma_rhs_bytes(const MfmaPack& pk, int k);
adasap_status_t mfma_pack_rhs(const MfmaPack& pk, const void* Z, DT zt, int k, void* zpack,
                              hipStream_t s);
// G = K(X[B], X) Z + epilogue (rows of the packed point set selected by B)
adasap_status_t mfma_kblock_rows(const MfmaPack& pk, int kern, double ell, int prec,
                                 const int64_t* B, int64_t b, const void* zpack, const void* Z,
                                 DT zt, int k, void* out, const KbEpilogue& ep, DevBuf& part,
                                 hipStream_t s);
// OUT = K(Xr, X) Z for arbitrary query points Xr (m x d, type xt); output type ot
adasap_status_t mfma_kblock_points(const MfmaPack& pk, int kern, double ell, const void* Xr,
                                   DT xt, int64_t m, const void* zpack, int k, void* out, DT ot,
                                   DevBuf& part, hipStream_t s);
// residual rows: OUT = K(X, X) W + epilogue, float64 accumulation
adasap_status_t mfma_residual(const MfmaPack& pk, int kern, double ell, const void* W, DT wt,
                              int k, void* out, const KbEpilogue& ep, DevBuf& part, DevBuf& tmp,
                              hipStream_t s);

}  // namespace adasap
