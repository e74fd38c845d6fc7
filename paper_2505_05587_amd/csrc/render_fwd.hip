// Stage 3: front-to-back alpha blending (Eq. alpha_blend) of every tile of
// every view in one persistent launch.
//
// A workgroup owns one screen tile at a time (one thread per pixel, each
// wavefront an 8x8 quadrant) and takes the next tile from a global atomic
// queue when done, so tiles with long instance lists do not stall the rest of
// the grid.  The tile's instances are staged through LDS in batches of one
// record per thread.  A wavefront skips an entry outright when its quadrant
// lies outside the entry's alpha >= alpha_min ellipse, stops when all its
// pixels are saturated, and the workgroup leaves the tile when every pixel's
// transmittance has hit the cut-off.
#include "common.h"

namespace sg {

template <int TW, int TH>
__global__ void __launch_bounds__(TW* TH) k_render_fwd(const steepgs_splat* __restrict__ splats,
                                                      const uint32_t* __restrict__ vals,
                                                      const uint32_t* __restrict__ ranges,
                                                      const steepgs_camera* __restrict__ cams, int V,
                                                      steepgs_opts opt, int total_tiles,
                                                      const float* __restrict__ target, float* __restrict__ image,
                                                      float* __restrict__ T_final, uint32_t* __restrict__ n_contrib,
                                                      uint32_t* __restrict__ n_used, float* __restrict__ loss,
                                                      uint32_t* __restrict__ queue) {
  constexpr int NT = TW * TH;
  constexpr int WX = TW / 8;          // each wavefront owns an 8x8 pixel quadrant of the tile
  __shared__ float4 s_m[NT];          // mean x, mean y, cut-off half extents x, y
  __shared__ float4 s_q[NT];          // conic a, b, c, opacity
  __shared__ float4 s_col[NT];        // rgb
  __shared__ float s_red[NT / 64];
  __shared__ int s_tile;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int qx = (wave % WX) * 8 + (lane & 7), qy = (wave / WX) * 8 + (lane >> 3);
  for (;;) {
    // The barrier closes the previous tile before lane 0 fetches the next one,
    // so no lane-0-only region can span the loop's back edge (the compiler
    // would otherwise merge them and let the other lanes re-enter the tile
    // loop without the fetch).
    __syncthreads();
    if (tid == 0) s_tile = (int)atomicAdd(queue, 1u);
    __syncthreads();
    // scalar (wave-uniform) copy: the loop exit below must be a uniform branch
    const int tile = __builtin_amdgcn_readfirstlane(s_tile);
    if (tile >= total_tiles) break;
    const int v = view_of_tile(cams, V, tile);
    const int W = cams[v].width, H = cams[v].height, tiles_x = cams[v].tiles_x;
    const int64_t pix_off = cams[v].pixel_offset;
    const int lt = tile - cams[v].tile_offset;
    const int tx0 = (lt % tiles_x) * TW, ty0 = (lt / tiles_x) * TH;
    const int px = tx0 + qx, py = ty0 + qy;
    const bool inside = px < W && py < H;
    // the wavefront's pixel block, for the per-wave cut-off test
    const float wx0 = (float)(tx0 + (wave % WX) * 8), wy0 = (float)(ty0 + (wave / WX) * 8);
    const float wx1 = wx0 + 7.f, wy1 = wy0 + 7.f;
    const uint32_t begin = ranges[2 * tile], end = ranges[2 * tile + 1];
    const float fx = (float)px, fy = (float)py;
    float T = 1.f, C0 = 0.f, C1 = 0.f, C2 = 0.f;
    uint32_t last = 0, used = 0;
    bool done = !inside;
    for (uint32_t b0 = begin; b0 < end; b0 += NT) {
      if (__builtin_amdgcn_readfirstlane(__syncthreads_count(done)) == NT) break;
      const uint32_t idx = b0 + tid;
      if (idx < end) {
        const steepgs_splat s = splats[vals[idx]];
        float ex, ey;
        cutoff_extent(s.conic_a, s.conic_b, s.conic_c, s.opacity, opt.alpha_min, ex, ey);
        s_m[tid] = make_float4(s.mean_x, s.mean_y, ex, ey);
        s_q[tid] = make_float4(s.conic_a, s.conic_b, s.conic_c, s.opacity);
        s_col[tid] = make_float4(s.rgb[0], s.rgb[1], s.rgb[2], 0.f);
      }
      __syncthreads();
      const int cnt = (int)min((uint32_t)NT, end - b0);
      for (int j = 0; j < cnt; ++j) {
        if (ballot(!done) == 0) break;  // the whole wavefront is finished
        const float4 m = s_m[j];
        // no pixel of this wavefront reaches alpha_min: skip for the whole wave
        const bool hit = (m.x + m.z >= wx0) && (m.x - m.z <= wx1) && (m.y + m.w >= wy0) && (m.y - m.w <= wy1);
        if (!__builtin_amdgcn_readfirstlane((int)hit)) continue;
        if (done) continue;
        const float4 q = s_q[j];
        const float dx = fx - m.x, dy = fy - m.y;
        const float G = __expf(splat_power(dx, dy, q.x, q.y, q.z));
        const float alpha = fminf(opt.alpha_max, q.w * G);
        if (alpha < opt.alpha_min) continue;
        const float Tn = T * (1.f - alpha);
        if (Tn < opt.t_min) {
          done = true;
          continue;
        }
        const float4 c = s_col[j];
        const float w = alpha * T;
        C0 += c.x * w;
        C1 += c.y * w;
        C2 += c.z * w;
        T = Tn;
        last = b0 - begin + (uint32_t)j + 1u;
        ++used;
      }
    }
    float err = 0.f;
    if (inside) {
      const int64_t p = pix_off + (int64_t)py * W + px;
      const int64_t plane = (int64_t)W * H;
      float* img = image + 3 * pix_off + (int64_t)py * W + px;
      const float o0 = C0 + T * opt.bg[0], o1 = C1 + T * opt.bg[1], o2 = C2 + T * opt.bg[2];
      img[0] = o0;
      img[plane] = o1;
      img[2 * plane] = o2;
      T_final[p] = T;
      n_contrib[p] = last;
      if (n_used) n_used[p] = used;
      if (target) {
        const float* tg = target + 3 * pix_off + (int64_t)py * W + px;
        err = fabsf(o0 - tg[0]) + fabsf(o1 - tg[plane]) + fabsf(o2 - tg[2 * plane]);
      }
    }
    if (target) {
      err = wave_sum_dpp(err);
      if (lane == 0) s_red[wave] = err;
      __syncthreads();
      if (tid == 0) {
        float s = 0.f;
        for (int w = 0; w < NT / 64; ++w) s += s_red[w];
        atomicAdd(&loss[v], s / (3.f * (float)W * (float)H));
      }
    }
  }
}

__global__ void k_zero_f32(float* __restrict__ p, int64_t count) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = 0.f;
}

__global__ void k_zero_u32(uint32_t* __restrict__ p, int64_t count) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = 0u;
}

size_t render_fwd_workspace() { return 256; }

template <int TW, int TH>
static void launch_fwd(int grid, hipStream_t st, const steepgs_splat* splats, const uint32_t* vals,
                       const uint32_t* ranges, const steepgs_camera* cams, int V, const steepgs_opts& opt,
                       int total_tiles, const float* target, float* image, float* T_final, uint32_t* n_contrib,
                       uint32_t* n_used, float* loss, uint32_t* queue) {
  hipLaunchKernelGGL((k_render_fwd<TW, TH>), dim3(grid), dim3(TW * TH), 0, st, splats, vals, ranges, cams, V, opt,
                     total_tiles, target, image, T_final, n_contrib, n_used, loss, queue);
}

}  // namespace sg

using namespace sg;

extern "C" steepgs_status steepgs_render_fwd(const steepgs_splat* d_splats, int64_t n, const uint32_t* d_vals,
                                             const uint32_t* d_tile_ranges, const steepgs_camera* d_cams, int32_t V,
                                             const steepgs_opts* opts, int32_t total_tiles, int64_t total_pixels,
                                             const float* d_target, float* d_image, float* d_T_final,
                                             uint32_t* d_n_contrib, uint32_t* d_n_used, float* d_loss, void* d_ws,
                                             size_t ws_bytes,
                                             void* stream) {
  if (n < 0 || V <= 0 || total_tiles <= 0 || total_pixels <= 0 || !opts_ok(opts)) return STEEPGS_ERR_INVALID_ARG;
  if (!d_tile_ranges || !d_cams || !d_image || !d_T_final || !d_n_contrib) return STEEPGS_ERR_INVALID_ARG;
  if (d_target && !d_loss) return STEEPGS_ERR_INVALID_ARG;
  if (!d_ws || ws_bytes < render_fwd_workspace()) return STEEPGS_ERR_WORKSPACE;
  hipStream_t st = as_stream(stream);
  uint32_t* queue = static_cast<uint32_t*>(d_ws);
  hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, st, queue, (int64_t)1);
  if (d_target) hipLaunchKernelGGL(k_zero_f32, dim3((unsigned)ceil_div(V, 64)), dim3(64), 0, st, d_loss, (int64_t)V);
  const int grid = (int)std::min<int64_t>(total_tiles, (int64_t)device_cu_count() * 8);
  const steepgs_opts& o = *opts;
  timer_begin(STEEPGS_TIMER_RENDER_FWD, st);
  if (o.tile_w == 16 && o.tile_h == 16)
    launch_fwd<16, 16>(grid, st, d_splats, d_vals, d_tile_ranges, d_cams, V, o, total_tiles, d_target, d_image,
                       d_T_final, d_n_contrib, d_n_used, d_loss, queue);
  else if (o.tile_w == 16 && o.tile_h == 8)
    launch_fwd<16, 8>(grid, st, d_splats, d_vals, d_tile_ranges, d_cams, V, o, total_tiles, d_target, d_image,
                      d_T_final, d_n_contrib, d_n_used, d_loss, queue);
  else
    launch_fwd<8, 8>(grid, st, d_splats, d_vals, d_tile_ranges, d_cams, V, o, total_tiles, d_target, d_image,
                     d_T_final, d_n_contrib, d_n_used, d_loss, queue);
  timer_end(STEEPGS_TIMER_RENDER_FWD, st);
  SG_TRY_LAUNCH();
  return STEEPGS_OK;
}
