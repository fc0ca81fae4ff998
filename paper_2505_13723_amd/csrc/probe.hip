// Instruction-rate probe of the part the library runs on (for the rooflines of the
// measurement, not a step of the method): register-only loops of one instruction kind, with
// enough independent chains per wave and waves per SIMD to reach the issue rate.
//   exp  : v_exp_f32 (the transcendental of every kernel value)
//   valu : v_fma_f32 (a full-rate vector instruction)
//   mfma : v_mfma_f32_32x32x16_f16 with four independent accumulators per wave
#include "internal.h"

namespace adasap {

namespace {

typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef float f16v __attribute__((ext_vector_type(16)));

constexpr int PROBE_WG = 2048;  // 8 workgroups of 256 per CU on 256 CUs
constexpr int PROBE_CHAINS = 16;

__global__ __launch_bounds__(256) void probe_exp_kernel(float* out, int iters) {
  float x[PROBE_CHAINS];
#pragma unroll
  for (int i = 0; i < PROBE_CHAINS; ++i) x[i] = 0.001f * (float)(threadIdx.x + i);
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int i = 0; i < PROBE_CHAINS; ++i) x[i] = __builtin_amdgcn_exp2f(-x[i]);
  }
  float s = 0.0f;
#pragma unroll
  for (int i = 0; i < PROBE_CHAINS; ++i) s += x[i];
  out[blockIdx.x * 256 + threadIdx.x] = s;
}

__global__ __launch_bounds__(256) void probe_fma_kernel(float* out, int iters, float a, float b) {
  float x[PROBE_CHAINS];
#pragma unroll
  for (int i = 0; i < PROBE_CHAINS; ++i) x[i] = 0.001f * (float)(threadIdx.x + i);
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int i = 0; i < PROBE_CHAINS; ++i) x[i] = __builtin_fmaf(x[i], a, b);
  }
  float s = 0.0f;
#pragma unroll
  for (int i = 0; i < PROBE_CHAINS; ++i) s += x[i];
  out[blockIdx.x * 256 + threadIdx.x] = s;
}

__global__ __launch_bounds__(256) void probe_mfma_kernel(float* out, int iters) {
  half8 a, b;
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    a[i] = (_Float16)(0.001f * (float)(threadIdx.x + i));
    b[i] = (_Float16)(0.002f * (float)i);
  }
  f16v c0 = {}, c1 = {}, c2 = {}, c3 = {};
  for (int it = 0; it < iters; ++it) {
    c0 = __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c0, 0, 0, 0);
    c1 = __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c1, 0, 0, 0);
    c2 = __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c2, 0, 0, 0);
    c3 = __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c3, 0, 0, 0);
  }
  float s = 0.0f;
#pragma unroll
  for (int i = 0; i < 16; ++i) s += c0[i] + c1[i] + c2[i] + c3[i];
  out[blockIdx.x * 256 + threadIdx.x] = s;
}

}  // namespace
}  // namespace adasap

using namespace adasap;

extern "C" adasap_status_t adasap_probe_rates(void* stream, double* out) {
  if (!out) {
    set_error("out must be a host array of 3 doubles");
    return ADASAP_ERR_INVALID_ARG;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  int dev = 0, cus = 256;
  ADASAP_HIP(hipGetDevice(&dev));
  ADASAP_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  DevBuf buf;
  ADASAP_TRY(buf.ensure((size_t)PROBE_WG * 256 * sizeof(float)));
  hipEvent_t e0 = nullptr, e1 = nullptr;
  ADASAP_HIP(hipEventCreate(&e0));
  ADASAP_HIP(hipEventCreate(&e1));
  struct EvFree {
    hipEvent_t a, b;
    ~EvFree() {
      if (a) (void)hipEventDestroy(a);
      if (b) (void)hipEventDestroy(b);
    }
  } evf{e0, e1};
  float* o = buf.as<float>();
  const int iters = 4000;
  // one warm-up and one timed launch of each; ms of the timed launch
  auto timed = [&](int which, float& ms) -> adasap_status_t {
    for (int rep = 0; rep < 2; ++rep) {
      if (rep == 1) ADASAP_HIP(hipEventRecord(e0, s));
      if (which == 0) hipLaunchKernelGGL(probe_exp_kernel, dim3(PROBE_WG), dim3(256), 0, s, o, iters);
      else if (which == 1) hipLaunchKernelGGL(probe_fma_kernel, dim3(PROBE_WG), dim3(256), 0, s, o, iters, 0.999f, 0.001f);
      else hipLaunchKernelGGL(probe_mfma_kernel, dim3(PROBE_WG), dim3(256), 0, s, o, iters);
      ADASAP_LAUNCH_CHECK();
    }
    ADASAP_HIP(hipEventRecord(e1, s));
    ADASAP_HIP(hipEventSynchronize(e1));
    ADASAP_HIP(hipEventElapsedTime(&ms, e0, e1));
    return ADASAP_OK;
  };
  float ms[3];
  for (int w = 0; w < 3; ++w) ADASAP_TRY(timed(w, ms[w]));
  const double waves = PROBE_WG * 4.0, simds = cus * 4.0;
  // ns per wave instruction per SIMD (exp, fma); float16 32x32x16 TFLOP/s over the part
  out[0] = ms[0] * 1e6 / (waves * iters * PROBE_CHAINS / simds);
  out[1] = ms[1] * 1e6 / (waves * iters * PROBE_CHAINS / simds);
  out[2] = waves * iters * 4.0 * 32768.0 / (ms[2] * 1e-3) / 1e12;
  return ADASAP_OK;
}
