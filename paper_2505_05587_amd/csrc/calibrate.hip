// Measurement support: the achievable vector-ALU rate of the device.
//
// Every lane runs kChains independent fp32 fused multiply-add chains for
// `iters` steps (plain v_fma_f32, no packed-FP32 instructions, like every
// kernel of this library), so the only limit is the VALU issue rate.  The
// chains converge (|a| < 1), and their sum is stored so that no step can be
// dropped.  Flops = blocks * 256 * iters * kChains * 2.
#include "common.h"

namespace sg {

constexpr int kCalChains = 8;

__global__ void __launch_bounds__(256) k_fma_loop(float* __restrict__ out, int iters, float a, float b) {
  const int tid = blockIdx.x * blockDim.x + threadIdx.x;
  float x[kCalChains];
#pragma unroll
  for (int k = 0; k < kCalChains; ++k) x[k] = (float)(tid & 255) * 1e-3f + (float)k;
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int k = 0; k < kCalChains; ++k) x[k] = __builtin_fmaf(x[k], a, b);
  }
  float s = 0.f;
#pragma unroll
  for (int k = 0; k < kCalChains; ++k) s += x[k];
  out[tid] = s;
}

}  // namespace sg

using namespace sg;

extern "C" steepgs_status steepgs_calibrate_valu(float* d_out, int32_t blocks, int32_t iters, void* stream) {
  if (!d_out || blocks <= 0 || iters <= 0) return STEEPGS_ERR_INVALID_ARG;
  hipLaunchKernelGGL(k_fma_loop, dim3((unsigned)blocks), dim3(256), 0, as_stream(stream), d_out, iters, 0.999f, 1e-3f);
  SG_TRY_LAUNCH();
  return STEEPGS_OK;
}
