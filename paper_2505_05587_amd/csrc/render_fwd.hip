// Stage 3: front-to-back alpha blending (Eq. alpha_blend) of every tile of
// every view in one persistent launch.
//
// A workgroup owns one screen tile at a time (one thread per pixel, each
// wavefront an 8x8 quadrant) and takes the next tile from a global atomic
// queue when done, so tiles with long instance lists do not stall the rest of
// the grid.  The tile's instances are staged through LDS in batches of one
// record per thread; the loading thread also tests the entry's cut-off box
// against every quadrant, and each wavefront then walks only the entries
// that reach its quadrant (a per-chunk bit mask scanned on the scalar unit).
// A wavefront stops when all its pixels are saturated, and the workgroup
// leaves the tile when every pixel's transmittance has hit the cut-off.
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
  constexpr int NW = NT / 64;         // wavefronts per workgroup = 64-entry chunks per batch
  constexpr int WX = TW / 8;          // each wavefront owns an 8x8 pixel quadrant of the tile
  __shared__ float4 s_a[NT];          // mean x, mean y, conic a, conic b
  __shared__ float4 s_c[NT];          // conic c, opacity, red, green
  __shared__ float s_bl[NT];          // blue
  __shared__ uint64_t s_bits[NW][NW]; // [wave][chunk]: entries of the chunk that reach the wave's quadrant
  __shared__ float s_red[NW];
  __shared__ int s_tile;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int qx = (wave % WX) * 8 + (lane & 7), qy = (wave / WX) * 8 + (lane >> 3);
  const float cut = footprint_power_cut(opt);
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
    const uint32_t begin = ranges[2 * tile], end = ranges[2 * tile + 1];
    const float fx = (float)px, fy = (float)py;
    float T = 1.f, C0 = 0.f, C1 = 0.f, C2 = 0.f;
    uint32_t last = 0, used = 0;
    bool done = !inside;
    for (uint32_t b0 = begin; b0 < end; b0 += NT) {
      if (__builtin_amdgcn_readfirstlane(__syncthreads_count(done)) == NT) break;
      // stage one batch; the thread that loads an entry tests its cut-off
      // box (alpha >= alpha_min and inside the footprint) against the
      // quadrant of every wavefront
      const uint32_t idx = b0 + tid;
      uint32_t qmask = 0;
      if (idx < end) {
        const steepgs_splat s = splats[vals[idx]];
        float ex, ey;
        cutoff_extent(s.conic_a, s.conic_b, s.conic_c, s.opacity, opt, ex, ey);
        s_a[tid] = make_float4(s.mean_x, s.mean_y, s.conic_a, s.conic_b);
        s_c[tid] = make_float4(s.conic_c, s.opacity, s.rgb[0], s.rgb[1]);
        s_bl[tid] = s.rgb[2];
#pragma unroll
        for (int w = 0; w < NW; ++w) {
          const float x0 = (float)(tx0 + (w % WX) * 8), y0 = (float)(ty0 + (w / WX) * 8);
          const bool hit = (s.mean_x + ex >= x0) && (s.mean_x - ex <= x0 + 7.f) && (s.mean_y + ey >= y0) &&
                           (s.mean_y - ey <= y0 + 7.f);
          qmask |= hit ? (1u << w) : 0u;
        }
      }
#pragma unroll
      for (int w = 0; w < NW; ++w) {
        const uint64_t b = ballot((qmask >> w) & 1u);
        if (lane == 0) s_bits[w][wave] = b;
      }
      __syncthreads();
      // this wavefront's entries of the batch, front to back
      for (int c = 0; c < NW; ++c) {
        uint64_t bits = uniform_u64(s_bits[wave][c]);
        while (bits) {
          if (ballot(!done) == 0) break;  // the whole wavefront is finished
          const int j = c * 64 + (int)__builtin_ctzll(bits);
          bits &= bits - 1;
          const float4 a = s_a[j];
          const float4 q = s_c[j];
          if (done) continue;
          const float dx = fx - a.x, dy = fy - a.y;
          const float power = splat_power(dx, dy, a.z, a.w, q.x);
          if (power < cut) continue;  // outside the footprint
          const float alpha = fminf(opt.alpha_max, q.y * __expf(power));
          if (alpha < opt.alpha_min) continue;
          const float Tn = T * (1.f - alpha);
          if (Tn < opt.t_min) {
            done = true;
            continue;
          }
          const float w = alpha * T;
          C0 += q.z * w;
          C1 += q.w * w;
          C2 += s_bl[j] * w;
          T = Tn;
          last = b0 - begin + (uint32_t)j + 1u;
          ++used;
        }
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
        for (int w = 0; w < NW; ++w) s += s_red[w];
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
