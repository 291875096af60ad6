// Roofline calibration of the bf16 matrix cores (measurement support; no
// part of the method).
//
// The split-precision gradient kernel issues v_mfma_f32_32x32x16_bf16
// products on operands whose bits look random (the hi and lo planes of X, of
// Theta and of the residuals).  The chip holds its power limit by lowering
// its clock, and the power of a matrix product grows with the switching
// activity of its operands, so the rate a bf16 MFMA kernel can sustain
// depends on the data it multiplies.  k_calib_mfma keeps every SIMD's matrix
// core busy (two waves per SIMD, operands read from LDS as in the gradient
// kernel, one MFMA chain per operand pair) on either constant operands or
// seeded random bf16 operands; the two rates bracket what the gradient
// kernel's products can reach on this part.
#include <hip/hip_runtime.h>

#include "pcv_internal.h"

namespace pcv {
namespace {

typedef __bf16 cbf16x8 __attribute__((ext_vector_type(8)));
typedef float cf32x16 __attribute__((ext_vector_type(16)));

constexpr int CAL_WORDS = 6144;        // 96 KB of uint4: one 8-wave workgroup per CU
constexpr int CAL_ITERS = 2000;
constexpr int CAL_MFMA_PER_ITER = 16;  // per wave

__device__ __forceinline__ uint32_t cal_hash(uint32_t x) {
  x ^= x >> 16;
  x *= 0x7feb352du;
  x ^= x >> 15;
  x *= 0x846ca68bu;
  x ^= x >> 16;
  return x;
}

// bf16 bits with random sign and mantissa and a binary exponent in [-8, -1]
// (magnitudes in [2^-8, 1)), the range of the split kernel's operands
__device__ __forceinline__ uint32_t cal_bf16(uint32_t h) { return (h & 0x807fu) | ((119u + (h >> 8) % 8u) << 7); }

__global__ __launch_bounds__(512) void k_calib_mfma(int random, float* out) {
  __shared__ uint4 buf[CAL_WORDS];
  const int tid = threadIdx.x, lane = tid & 63;
  for (int i = tid; i < CAL_WORDS; i += 512) {
    uint32_t w[4];
    for (int j = 0; j < 4; ++j) {
      const uint32_t h = cal_hash(static_cast<uint32_t>(i * 4 + j) + 12345u * (blockIdx.x + 1));
      w[j] = random ? (cal_bf16(h) | (cal_bf16(cal_hash(h)) << 16)) : 0x3f803f80u;   // 1.0 pairs
    }
    buf[i] = uint4{w[0], w[1], w[2], w[3]};
  }
  __syncthreads();
  cf32x16 c0 = {}, c1 = {};
  for (int it = 0; it < CAL_ITERS; ++it) {
#pragma unroll
    for (int f = 0; f < CAL_MFMA_PER_ITER / 2; ++f) {
      // 32 operand pairs of 128 words cycle through words [0, 4096)
      const int base = ((it * (CAL_MFMA_PER_ITER / 2) + f) & 31) * 128;
      const cbf16x8 a = __builtin_bit_cast(cbf16x8, buf[base + lane]);
      const cbf16x8 b = __builtin_bit_cast(cbf16x8, buf[base + 64 + lane]);
      c0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c0, 0, 0, 0);
      c1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(b, a, c1, 0, 0, 0);
    }
  }
  float s = 0.f;
#pragma unroll
  for (int i = 0; i < 16; ++i) s += c0[i] + c1[i];
  out[blockIdx.x * 512 + tid] = s;
}

}  // namespace
}  // namespace pcv

extern "C" {

pcv_status pcv_calib_mfma(int32_t data_kind, int32_t launches, double* tflops) {
  if ((data_kind != 0 && data_kind != 1) || launches < 1 || !tflops) return PCV_ERR_INVALID_ARG;
  int dev = 0, n_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n_cu < 1)
    return PCV_ERR_DEVICE;
  float* out = nullptr;
  if (hipMalloc(&out, sizeof(float) * 512 * n_cu) != hipSuccess) return PCV_ERR_NOMEM;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  if (e == hipSuccess) {
    // one untimed launch, then the timed ones back to back on the null stream
    hipLaunchKernelGGL(pcv::k_calib_mfma, dim3(n_cu), dim3(512), 0, nullptr, data_kind, out);
    e = hipEventRecord(e0, nullptr);
  }
  for (int r = 0; e == hipSuccess && r < launches; ++r) {
    hipLaunchKernelGGL(pcv::k_calib_mfma, dim3(n_cu), dim3(512), 0, nullptr, data_kind, out);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipEventRecord(e1, nullptr);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  float ms = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipFree(out);
  if (e != hipSuccess || ms <= 0.f) return PCV_ERR_DEVICE;
  // 8 waves per workgroup, one workgroup per CU; 2 * 32 * 32 * 16 flops per product
  const double flops = static_cast<double>(n_cu) * 8 * pcv::CAL_ITERS * pcv::CAL_MFMA_PER_ITER * 32768.0 * launches;
  *tflops = flops / (ms * 1e-3) * 1e-12;
  return PCV_OK;
}

}  // extern "C"
