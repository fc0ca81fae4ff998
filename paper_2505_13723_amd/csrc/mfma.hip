// Matrix-core kernel-block products (placeholder until the gfx950 kernels land).
#include "mfma.h"

namespace adasap {

static adasap_status_t unsupported() {
  set_error("MIXED precision kernels are not built yet");
  return ADASAP_ERR_UNSUPPORTED;
}

size_t mfma_pack_bytes(int64_t, int, int) { return 0; }
adasap_status_t mfma_pack_create(MfmaPack&, int64_t, int, int, const void*, DT, int, double,
                                 hipStream_t) { return unsupported(); }
size_t mfma_rhs_bytes(const MfmaPack&, int) { return 16; }
adasap_status_t mfma_pack_rhs(const MfmaPack&, const void*, DT, int, void*, hipStream_t) { return unsupported(); }
adasap_status_t mfma_kblock_rows(const MfmaPack&, int, double, int, const int64_t*, int64_t,
                                 const void*, const void*, DT, int, void*, const KbEpilogue&,
                                 DevBuf&, hipStream_t) { return unsupported(); }
adasap_status_t mfma_kblock_points(const MfmaPack&, int, double, const void*, DT, int64_t,
                                   const void*, int, void*, DT, DevBuf&, hipStream_t) { return unsupported(); }
adasap_status_t mfma_residual(const MfmaPack&, int, double, const void*, DT, int, void*,
                              const KbEpilogue&, DevBuf&, DevBuf&, hipStream_t) { return unsupported(); }

}  // namespace adasap
