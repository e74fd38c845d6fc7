// Training-loop support around the hot path (Algorithm 1): the Adam step of
// the 3DGS training pipeline the paper keeps (Sec. 5.1), and the remapping of
// per-Gaussian optimizer state onto the layout a densification produced.
#include "common.h"
#include "scan.h"

namespace sg {

// learning-rate group of a parameter row
SG_DEV int adam_group(int row) {
  if (row < STEEPGS_ROW_LOG_SCALE) return 0;  // position
  if (row < STEEPGS_ROW_QUAT) return 1;       // log-scales
  if (row < STEEPGS_ROW_OPACITY) return 2;    // quaternion
  if (row < STEEPGS_ROW_SH) return 3;         // opacity logit
  if (row < STEEPGS_ROW_SH + 3) return 4;     // SH degree 0
  return 5;                                   // SH degrees >= 1
}

__global__ void k_step_inc(int64_t* step) { *step += 1; }

// one thread per parameter element; rows are contiguous in the planar layout
__global__ void __launch_bounds__(256) k_adam(float* __restrict__ p, const float* __restrict__ g,
                                              float* __restrict__ m, float* __restrict__ v, int64_t n, int F,
                                              steepgs_adam_opts o, const int64_t* __restrict__ step,
                                              float* __restrict__ G) {
  const double t = (double)*step;
  const float bc1 = (float)(1.0 - pow((double)o.beta1, t));
  const float sbc2 = sqrtf((float)(1.0 - pow((double)o.beta2, t)));
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < (int64_t)F * n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int row = (int)(e / n);
    const float gi = g[e];
    if (G && row < 3) G[e] += gi;  // Algorithm 1's accumulated position gradient
    const float mi = o.beta1 * m[e] + (1.f - o.beta1) * gi;
    const float vi = o.beta2 * v[e] + (1.f - o.beta2) * gi * gi;
    m[e] = mi;
    v[e] = vi;
    const float denom = sqrtf(vi) / sbc2 + o.eps;
    p[e] -= (o.lr[adam_group(row)] / bc1) * (mi / denom);
  }
}

// Gabs[i] += |dL/dp_i| (the position rows 0-2 of one Gaussian)
__global__ void __launch_bounds__(256) k_grad_norm(const float* __restrict__ g, int64_t n, float* __restrict__ Gabs) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float x = g[i], y = g[n + i], z = g[2 * n + i];
  Gabs[i] += sqrtf(x * x + y * y + z * z);
}

struct LoadSplit {
  const uint8_t* f;
  SG_DEV uint32_t operator()(int64_t i) const { return f[i] ? 1u : 0u; }
};

// dst[r][i + before_i] = src[r][i] for a kept Gaussian; both slots of a split
// one start from zero
__global__ void __launch_bounds__(256) k_split_remap(const float* __restrict__ src, int rows, int64_t n,
                                                     const uint8_t* __restrict__ split,
                                                     const uint32_t* __restrict__ before, float* __restrict__ dst,
                                                     int64_t cap) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t o = i + (int64_t)before[i];
  const bool s = split[i] != 0;
  if (o + (s ? 1 : 0) >= cap) return;
  for (int r = 0; r < rows; ++r) {
    dst[(int64_t)r * cap + o] = s ? 0.f : src[(int64_t)r * n + i];
    if (s) dst[(int64_t)r * cap + o + 1] = 0.f;
  }
}

}  // namespace sg

using namespace sg;

extern "C" steepgs_status steepgs_adam_step(float* d_params, const float* d_grads, float* d_m, float* d_v, int64_t n,
                                            int32_t sh_degree, const steepgs_adam_opts* opts, int64_t* d_step,
                                            float* d_G, float* d_Gabs, void* stream) {
  if (n < 0 || sh_degree < 0 || sh_degree > 3 || !opts || !d_step) return STEEPGS_ERR_INVALID_ARG;
  if (!(opts->beta1 >= 0.f && opts->beta1 < 1.f && opts->beta2 >= 0.f && opts->beta2 < 1.f && opts->eps > 0.f))
    return STEEPGS_ERR_INVALID_ARG;
  if (n > 0 && (!d_params || !d_grads || !d_m || !d_v)) return STEEPGS_ERR_INVALID_ARG;
  hipStream_t st = as_stream(stream);
  hipLaunchKernelGGL(k_step_inc, dim3(1), dim3(1), 0, st, d_step);
  if (n > 0) {
    const int F = STEEPGS_NUM_PARAMS(sh_degree);
    if (d_Gabs)
      hipLaunchKernelGGL(k_grad_norm, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, st, d_grads, n, d_Gabs);
    hipLaunchKernelGGL(k_adam, dim3(stride_grid((int64_t)F * n, 256)), dim3(256), 0, st, d_params, d_grads,
                       d_m, d_v, n, F, *opts, d_step, d_G);
  }
  SG_TRY_LAUNCH();
  return STEEPGS_OK;
}

extern "C" steepgs_status steepgs_split_remap(const float* d_src, int32_t rows, int64_t n, const uint8_t* d_split,
                                              float* d_dst, int64_t dst_capacity, void* d_ws, size_t ws_bytes,
                                              void* stream) {
  if (rows < 0 || n < 0 || dst_capacity < 0) return STEEPGS_ERR_INVALID_ARG;
  if (n == 0 || rows == 0) return STEEPGS_OK;
  if (!d_src || !d_split || !d_dst) return STEEPGS_ERR_INVALID_ARG;
  if (n >= (int64_t)1 << 31) return STEEPGS_ERR_INVALID_ARG;
  Carver c(d_ws);
  uint32_t* before = c.take<uint32_t>(n);
  uint32_t* partials = c.take<uint32_t>(scan_partials_count(n) + 1);
  if (!d_ws || ws_bytes < c.used + 256) return STEEPGS_ERR_WORKSPACE;
  hipStream_t st = as_stream(stream);
  if (exclusive_scan<LoadSplit, uint32_t, uint32_t>(LoadSplit{d_split}, n, before, partials, st) != hipSuccess)
    return STEEPGS_ERR_HIP;
  hipLaunchKernelGGL(k_split_remap, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, st, d_src, rows, n, d_split,
                     before, d_dst, dst_capacity);
  SG_TRY_LAUNCH();
  return STEEPGS_OK;
}
