// Stage 3: front-to-back alpha blending (Eq. alpha_blend) of every tile of
// every view in one persistent launch.
//
// One wavefront owns one screen tile at a time and takes the next tile from a
// global atomic queue when done, so tiles with long instance lists do not
// stall the rest of the grid; each lane owns one pixel in every 8x8 quadrant
// of the tile.  The tile's instances are staged through the wavefront's LDS
// slice in batches of 64; the loading lane tests the entry's cut-off region
// (alpha >= alpha_min inside the footprint: its bounding box, then the
// ellipse itself) against every quadrant, and a quadrant the entry cannot
// reach (or whose pixels are all saturated) is skipped for the whole
// wavefront.  The wavefront leaves the tile when every pixel's
// transmittance has hit the cut-off.
#include <mutex>

#include "common.h"

namespace sg {

// COUNT: also count each pixel's contributors (the optional n_used output);
// WAVES wavefronts per workgroup, each on a tile of its own
// Occupancy target of the blend kernels (wavefronts per SIMD), which sets
// their register budget (a build option: 512 / target registers per lane)
#ifndef SG_FWD_WAVES_PER_EU
#define SG_FWD_WAVES_PER_EU 6
#endif

template <int TW, int TH, bool COUNT, int WAVES>
__global__ void __launch_bounds__(64 * WAVES) __attribute__((amdgpu_waves_per_eu(SG_FWD_WAVES_PER_EU))) k_render_fwd(const steepgs_splat* __restrict__ splats,
                                                               const uint32_t* __restrict__ vals,
                                                               const uint32_t* __restrict__ ranges,
                                                               const steepgs_camera* __restrict__ cams, int V,
                                                               steepgs_opts opt, int total_tiles,
                                                               const float* __restrict__ target,
                                                               float* __restrict__ image, float* __restrict__ T_final,
                                                               uint32_t* __restrict__ n_contrib,
                                                               uint32_t* __restrict__ n_used, float* __restrict__ loss,
                                                               uint32_t* __restrict__ queue) {
  constexpr int NQ = TW * TH / 64;  // 8x8 quadrants of the tile = pixels per lane
  constexpr int QX = TW / 8;
  __shared__ float4 s_a[WAVES][64];  // float32 mean x, y, long axis x, y
  __shared__ float4 s_c[WAVES][64];  // e_long, e_short, opacity, red
  __shared__ float4 s_b[WAVES][64];  // green, blue, remainder constants cl, cs
  __shared__ float s_t[WAVES][64];   // smallest power2 taken (entry_power2_min)
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int lx = lane & 7, ly = lane >> 3;
  float4* const A = s_a[wave];
  float4* const Cq = s_c[wave];
  float4* const Bl = s_b[wave];
  float* const Th = s_t[wave];
  const float cut = footprint_power2_cut(opt);
  const int tmin_bits = __float_as_int(opt.t_min);
  for (;;) {
    // the wave barrier keeps the lane-0 fetch inside the loop
    __builtin_amdgcn_wave_barrier();
    uint32_t ticket = 0;
    if (lane == 0) ticket = atomicAdd(queue, 1u);
    const int tile = (int)__builtin_amdgcn_readfirstlane(ticket);
    if (tile >= total_tiles) break;
    const int v = view_of_tile(cams, V, tile);
    const int W = cams[v].width, H = cams[v].height, tiles_x = cams[v].tiles_x;
    const int64_t pix_off = cams[v].pixel_offset;
    const int lt = tile - cams[v].tile_offset;
    const int tx0 = (lt % tiles_x) * TW, ty0 = (lt / tiles_x) * TH;
    const uint32_t begin = ranges[2 * tile], end = ranges[2 * tile + 1];
    float T[NQ], C[NQ][3];
    uint32_t last[NQ], used[NQ];
    // per quadrant, the lanes whose pixel is finished (outside the image, or
    // stopped at the transmittance cut-off): wave-uniform lane masks
    uint64_t done[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int px = tx0 + (q % QX) * 8 + lx, py = ty0 + (q / QX) * 8 + ly;
      T[q] = 1.f;
      C[q][0] = C[q][1] = C[q][2] = 0.f;
      last[q] = used[q] = 0;
      done[q] = ballot(!(px < W && py < H));
    }
    for (uint32_t b0 = begin; b0 < end; b0 += 64) {
      // quadrants with a pixel still open (wave-uniform)
      uint32_t alive = 0;
#pragma unroll
      for (int q = 0; q < NQ; ++q) alive |= ~done[q] ? (1u << q) : 0u;
      alive = __builtin_amdgcn_readfirstlane(alive);
      if (!alive) break;
      // stage one batch of 64 entries in the wave's LDS slice; the loading
      // lane tests the entry's cut-off region (bounding box, then the
      // ellipse) against every quadrant
      const uint32_t idx = b0 + (uint32_t)lane;
      bool hitq[NQ];
#pragma unroll
      for (int q = 0; q < NQ; ++q) hitq[q] = false;
      __builtin_amdgcn_wave_barrier();
      if (idx < end) {
        const steepgs_splat sp = splats[vals[idx]];
        float ex, ey;
        cutoff_extent(sp.conic_a, sp.conic_b, sp.conic_c, sp.opacity, opt, ex, ey);
        const float lev = cutoff_level(sp.opacity, opt);
        const float ia = __builtin_amdgcn_rcpf(sp.conic_a), ic = __builtin_amdgcn_rcpf(sp.conic_c);
        const float2 rc = rem_axes(sp);
        A[lane] = make_float4(sp.mean_x, sp.mean_y, sp.axis_x, sp.axis_y);
        Cq[lane] = make_float4(sp.e_long, sp.e_short, sp.opacity, sp.rgb[0]);
        Bl[lane] = make_float4(sp.rgb[1], sp.rgb[2], rc.x, rc.y);
        Th[lane] = entry_power2_min(sp.opacity, cut, opt);
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
          const float x0 = (float)(tx0 + (q % QX) * 8), y0 = (float)(ty0 + (q / QX) * 8);
          hitq[q] = (sp.mean_x + ex >= x0) && (sp.mean_x - ex <= x0 + 7.f) && (sp.mean_y + ey >= y0) &&
                    (sp.mean_y - ey <= y0 + 7.f) &&
                    block_reach(sp.mean_x, sp.mean_y, sp.conic_a, sp.conic_b, sp.conic_c, ia, ic, lev, x0, y0,
                                x0 + 7.f, y0 + 7.f);
        }
      }
      uint64_t qm[NQ], any_q = 0;
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        qm[q] = ((alive >> q) & 1u) ? uniform_u64(ballot(hitq[q])) : 0ull;
        any_q |= qm[q];
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      // front to back over the batch
      while (any_q) {
        const int j = (int)__builtin_ctzll(any_q);
        any_q &= any_q - 1ull;
        const float4 a = A[j];
        const float4 cq = Cq[j];
        const float4 gb = Bl[j];  // green, blue, cl, cs
        const float pmin = Th[j];
        // the entry's 1-based position in the tile's list, in a vector
        // register once for all quadrants
        uint32_t pos1;
        asm volatile("v_mov_b32 %0, %1" : "=v"(pos1) : "s"(b0 - begin + (uint32_t)j + 1u));
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
          if (!((qm[q] >> j) & 1ull)) continue;  // wave-uniform
          // per pixel: predicated, no divergent branch
          const float dx = (float)(tx0 + (q % QX) * 8 + lx) - a.x;
          const float dy = (float)(ty0 + (q / QX) * 8 + ly) - a.y;
          const float power = splat_power2(dx, dy, a.z, a.w, gb.z, gb.w, cq.x, cq.y);
          const float alpha = fminf(opt.alpha_max, cq.z * __builtin_amdgcn_exp2f(power));
          const uint64_t in = ballot(power >= pmin) & ~done[q];
          // T after the entry: T - alpha T (the weight alpha T is needed anyway)
          const float wt = alpha * T[q];
          const float Tn = T[q] - wt;
          // else: would cross the cut-off, excluded, pixel done (Tn, t_min >= 0:
          // their float bits order as integers)
          const uint64_t keep = ballot(__float_as_int(Tn) >= tmin_bits);
          done[q] |= in & ~keep;
          const bool c = __builtin_amdgcn_inverse_ballot_w64(in & keep);
          // the weight is zero for a pixel that does not take the entry, so
          // the colour sums need no select (fma(colour, 0, C) = C)
          const float w = c ? wt : 0.f;
          C[q][0] += cq.w * w;
          C[q][1] += gb.x * w;
          C[q][2] += gb.y * w;
          T[q] = c ? Tn : T[q];
          last[q] = c ? pos1 : last[q];
          if (COUNT) used[q] += c ? 1u : 0u;
        }
      }
    }
    float err = 0.f;
    const int64_t plane = (int64_t)W * H;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int px = tx0 + (q % QX) * 8 + lx, py = ty0 + (q / QX) * 8 + ly;
      if (px < W && py < H) {
        const int64_t p = pix_off + (int64_t)py * W + px;
        float* img = image + 3 * pix_off + (int64_t)py * W + px;
        const float o0 = C[q][0] + T[q] * opt.bg[0], o1 = C[q][1] + T[q] * opt.bg[1], o2 = C[q][2] + T[q] * opt.bg[2];
        img[0] = o0;
        img[plane] = o1;
        img[2 * plane] = o2;
        T_final[p] = T[q];
        n_contrib[p] = last[q];
        if (COUNT) n_used[p] = used[q];
        if (target) {
          const float* tg = target + 3 * pix_off + (int64_t)py * W + px;
          err += fabsf(o0 - tg[0]) + fabsf(o1 - tg[plane]) + fabsf(o2 - tg[2 * plane]);
        }
      }
    }
    if (target) {
      err = wave_sum_dpp(err);
      if (lane == 0) atomicAdd(&loss[v], err / (3.f * (float)W * (float)H));
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

template <int TW, int TH, bool COUNT, int WAVES>
static void launch_fwd1(int grid, hipStream_t st, const steepgs_splat* splats, const uint32_t* vals,
                        const uint32_t* ranges, const steepgs_camera* cams, int V, const steepgs_opts& opt,
                        int total_tiles, const float* target, float* image, float* T_final, uint32_t* n_contrib,
                        uint32_t* n_used, float* loss, uint32_t* queue) {
  hipLaunchKernelGGL((k_render_fwd<TW, TH, COUNT, WAVES>), dim3(grid), dim3(64 * WAVES), 0, st, splats, vals, ranges,
                     cams, V, opt, total_tiles, target, image, T_final, n_contrib, n_used, loss, queue);
}

template <int TW, int TH>
static void launch_fwd(int grid, hipStream_t st, const steepgs_splat* splats, const uint32_t* vals,
                       const uint32_t* ranges, const steepgs_camera* cams, int V, const steepgs_opts& opt,
                       int total_tiles, const float* target, float* image, float* T_final, uint32_t* n_contrib,
                       uint32_t* n_used, float* loss, uint32_t* queue) {
#define SG_FWD(COUNT, WAVES)                                                                                       \
  launch_fwd1<TW, TH, COUNT, WAVES>(grid, st, splats, vals, ranges, cams, V, opt, total_tiles, target, image,     \
                                    T_final, n_contrib, n_used, loss, queue)
  const int w = raster_waves(opt);
  if (n_used) {
    if (w == 2) SG_FWD(true, 2); else if (w == 8) SG_FWD(true, 8); else SG_FWD(true, 4);
  } else {
    if (w == 2) SG_FWD(false, 2); else if (w == 8) SG_FWD(false, 8); else SG_FWD(false, 4);
  }
#undef SG_FWD
}

}  // namespace sg

using namespace sg;

static steepgs_status fwd_check(int64_t n, const uint32_t* d_tile_ranges, const steepgs_camera* d_cams, int32_t V,
                                const steepgs_opts* opts, int32_t total_tiles, int64_t total_pixels,
                                const float* d_target, float* d_image, float* d_T_final, uint32_t* d_n_contrib,
                                float* d_loss) {
  if (n < 0 || V <= 0 || total_tiles <= 0 || total_pixels <= 0 || !opts_ok(opts)) return STEEPGS_ERR_INVALID_ARG;
  if (!d_tile_ranges || !d_cams || !d_image || !d_T_final || !d_n_contrib) return STEEPGS_ERR_INVALID_ARG;
  if (d_target && !d_loss) return STEEPGS_ERR_INVALID_ARG;
  return STEEPGS_OK;
}

// queue: the persistent launch's tile counter (zeroed here by a kernel, so
// that the call stays legal under graph capture)
static steepgs_status fwd_launch(const steepgs_splat* d_splats, const uint32_t* d_vals, const uint32_t* d_tile_ranges,
                                 const steepgs_camera* d_cams, int32_t V, const steepgs_opts& o, int32_t total_tiles,
                                 const float* d_target, float* d_image, float* d_T_final, uint32_t* d_n_contrib,
                                 uint32_t* d_n_used, float* d_loss, uint32_t* queue, hipStream_t st) {
  hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, st, queue, (int64_t)1);
  if (d_target) hipLaunchKernelGGL(k_zero_f32, dim3((unsigned)ceil_div(V, 64)), dim3(64), 0, st, d_loss, (int64_t)V);
  const int grid = raster_grid(o, total_tiles);
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

extern "C" steepgs_status steepgs_render_fwd(const steepgs_splat* d_splats, int64_t n, const uint32_t* d_vals,
                                             const uint32_t* d_tile_ranges, const steepgs_camera* d_cams, int32_t V,
                                             const steepgs_opts* opts, int32_t total_tiles, int64_t total_pixels,
                                             const float* d_target, float* d_image, float* d_T_final,
                                             uint32_t* d_n_contrib, uint32_t* d_n_used, float* d_loss, void* d_ws,
                                             size_t ws_bytes,
                                             void* stream) {
  const steepgs_status chk = fwd_check(n, d_tile_ranges, d_cams, V, opts, total_tiles, total_pixels, d_target,
                                       d_image, d_T_final, d_n_contrib, d_loss);
  if (chk != STEEPGS_OK) return chk;
  if (!d_ws || ws_bytes < render_fwd_workspace()) return STEEPGS_ERR_WORKSPACE;
  return fwd_launch(d_splats, d_vals, d_tile_ranges, d_cams, V, raster_opts(*opts), total_tiles, d_target, d_image,
                    d_T_final, d_n_contrib, d_n_used, d_loss, static_cast<uint32_t*>(d_ws), as_stream(stream));
}

// ---------------------------------------------------------------------------
// Allocation-free variant.  Its scratch (the tile-queue counter) lives in a
// file-scope device array; each device holds its own copy, whose address is
// looked up once per device with that device current and kept on the host.
// Host code never passes the array's name to a kernel: it names a host-side
// stand-in, not device memory.

namespace sg {
constexpr size_t kNoAllocScratchBytes = 256;
constexpr int kNoAllocMaxDevices = 64;
static std::mutex g_noalloc_mu;
static uint32_t* g_noalloc_ptr[kNoAllocMaxDevices];
}  // namespace sg

static __device__ __align__(256) uint32_t scratch[sg::kNoAllocScratchBytes / sizeof(uint32_t)];

static steepgs_status noalloc_scratch(uint32_t** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0) return STEEPGS_ERR_HIP;
  if (dev >= kNoAllocMaxDevices) return STEEPGS_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lock(g_noalloc_mu);
  if (!g_noalloc_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return STEEPGS_ERR_HIP;
    g_noalloc_ptr[dev] = static_cast<uint32_t*>(p);
  }
  *out = g_noalloc_ptr[dev];
  return STEEPGS_OK;
}

extern "C" steepgs_status steepgs_render_fwd_noalloc(const steepgs_splat* d_splats, int64_t n, const uint32_t* d_vals,
                                                     const uint32_t* d_tile_ranges, const steepgs_camera* d_cams,
                                                     int32_t V, const steepgs_opts* opts, int32_t total_tiles,
                                                     int64_t total_pixels, const float* d_target, float* d_image,
                                                     float* d_T_final, uint32_t* d_n_contrib, uint32_t* d_n_used,
                                                     float* d_loss, void* stream) {
  const steepgs_status chk = fwd_check(n, d_tile_ranges, d_cams, V, opts, total_tiles, total_pixels, d_target,
                                       d_image, d_T_final, d_n_contrib, d_loss);
  if (chk != STEEPGS_OK) return chk;
  // the scratch a launch needs does not grow with the problem; a build whose
  // forward needed more than the array holds fails here, not on the device
  if (render_fwd_workspace() > kNoAllocScratchBytes) return STEEPGS_ERR_WORKSPACE;
  uint32_t* queue = nullptr;
  const steepgs_status st = noalloc_scratch(&queue);
  if (st != STEEPGS_OK) return st;
  return fwd_launch(d_splats, d_vals, d_tile_ranges, d_cams, V, raster_opts(*opts), total_tiles, d_target, d_image,
                    d_T_final, d_n_contrib, d_n_used, d_loss, queue, as_stream(stream));
}
