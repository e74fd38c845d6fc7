// Stage 1: projection of every Gaussian through every camera (Sec. 3,
// Eqs. sigma_3D and sigma_2D).  One thread per Gaussian loops over the V
// views, so the parameters are read from HBM once per batch, not once per
// view.
#include "projection.h"

namespace sg {

// One thread per Gaussian loops over the views; the Gaussian's SH
// coefficients are staged once in the thread's own LDS column, so every view
// reads them from LDS instead of HBM.  The per-view camera constants (centre,
// guard limits) are computed once per workgroup for a chunk of views.
constexpr int kProjThreads = 128;
constexpr int kCamChunk = 8;

template <int D>
__global__ void __launch_bounds__(kProjThreads) k_project(const float* __restrict__ params, int64_t n,
                                                          const steepgs_camera* __restrict__ cams, int V,
                                                          steepgs_opts opt, steepgs_splat* __restrict__ out,
                                                          uint32_t* __restrict__ tiles, uint32_t* __restrict__ dkeys) {
  constexpr int NS = 3 * (D + 1) * (D + 1);
  __shared__ float s_sh[NS * kProjThreads];  // [coefficient][thread]
  __shared__ double s_cc[kCamChunk * kCamConsts];
  const int tid = threadIdx.x;
  const int64_t i = (int64_t)blockIdx.x * kProjThreads + tid;
  const bool active = i < n;
  float* const sh = s_sh + tid;
  Gauss g;
  if (active) {
#pragma unroll
    for (int k = 0; k < NS; ++k) sh[k * kProjThreads] = params[(STEEPGS_ROW_SH + k) * n + i];
    load_gauss(params, n, i, g);
  }
  for (int v0 = 0; v0 < V; v0 += kCamChunk) {
    const int nv = min(kCamChunk, V - v0);
    __syncthreads();  // the previous chunk's constants are read by now
    if (tid < nv) camera_constants(cams[v0 + tid], opt, s_cc + tid * kCamConsts);
    __syncthreads();
    if (!active) continue;
    uint64_t near = 0;  // channels (3 per view of the chunk) within 1e-5 of the colour clamp
    for (int k = 0; k < nv; ++k) {
      const int v = v0 + k;
      const double* cc = s_cc + k * kCamConsts;
      CamD cam;
      load_cam(cc, cams[v], cam);
      ViewProj pv;
      const int64_t r = (int64_t)v * n + i;
      steepgs_splat s;
      uint32_t count = 0;
      float depth = 0.f;
      const double lim[2] = {cc[kCamLim], cc[kCamLim + 1]};
      if (project_view(g, cam, opt, lim, pv)) {
        const double campos[3] = {cc[kCamCentre], cc[kCamCentre + 1], cc[kCamCentre + 2]};
        const float pf[3] = {(float)g.p[0], (float)g.p[1], (float)g.p[2]};
        float rgb[3];
        near |= (uint64_t)view_colour<D>(pf, campos, sh, kProjThreads, rgb) << (3 * k);
        s.mean_x = (float)pv.mx;
        s.mean_y = (float)pv.my;
        s.mean_lo =
            half_bits((float)(pv.mx - (double)s.mean_x)) | (half_bits((float)(pv.my - (double)s.mean_y)) << 16);
        s.conic_a = (float)pv.A00;
        s.conic_b = (float)pv.A01;
        s.conic_c = (float)pv.A11;
        s.opacity = (float)g.o;
        s.rgb[0] = rgb[0];
        s.rgb[1] = rgb[1];
        s.rgb[2] = rgb[2];
        depth = (float)pv.pc[2];
        s.axis_x = (float)pv.ax;
        s.axis_y = (float)pv.ay;
        s.e_long = (float)(-0.72134752044448170368 * pv.lam_long);  // -log2(e) / 2
        s.e_short = (float)(-0.72134752044448170368 * pv.lam_short);
        s.rect_lo = (uint32_t)pv.rect[0] | ((uint32_t)pv.rect[1] << 16);
        s.rect_hi = (uint32_t)pv.rect[2] | ((uint32_t)pv.rect[3] << 16);
        // the rectangle's area: the sort's emission keeps the tiles that meet the footprint
        count = (uint32_t)((pv.rect[2] - pv.rect[0] + 1) * (pv.rect[3] - pv.rect[1] + 1));
      } else {
        s.mean_x = s.mean_y = 0.f;
        s.conic_a = s.conic_b = s.conic_c = 0.f;
        s.opacity = 0.f;
        s.rgb[0] = s.rgb[1] = s.rgb[2] = 0.f;
        s.mean_lo = 0u;
        s.axis_x = 1.f;
        s.axis_y = 0.f;
        s.e_long = s.e_short = 0.f;
        s.rect_lo = 1u;  // x0 = 1 > x1 = 0: empty
        s.rect_hi = 0u;
      }
      // four 16-byte stores
      float4* dst = reinterpret_cast<float4*>(out + r);
      const float4* src = reinterpret_cast<const float4*>(&s);
      dst[0] = src[0];
      dst[1] = src[1];
      dst[2] = src[2];
      dst[3] = src[3];
      tiles[r] = count;
      // the key of the sort's depth order: the float bits of the (positive)
      // depth, all ones for a culled record
      dkeys[r] = count ? __float_as_uint(depth) : 0xFFFFFFFFu;
    }
    // the channels too close to the clamp to call in fp32: fp64 in the
    // reference order decides and gives the value (rare; one call site)
    while (near) {
      const int b = __builtin_ctzll(near);
      near &= near - 1;
      const int k = b / 3, ch = b - 3 * k;
      const double c = colour_channel_fp64(params, n, i, D, s_cc + k * kCamConsts + kCamCentre, ch);
      out[(int64_t)(v0 + k) * n + i].rgb[ch] = c < 0.0 ? 0.f : (float)c;
    }
  }
}

}  // namespace sg

using namespace sg;

extern "C" steepgs_status steepgs_project(const float* d_params, int64_t n, int32_t sh_degree,
                                          const steepgs_camera* d_cams, int32_t V, const steepgs_opts* opts,
                                          steepgs_splat* d_splats, uint32_t* d_tiles_touched,
                                          uint32_t* d_depth_keys, void* stream) {
  if (n < 0 || V <= 0 || sh_degree < 0 || sh_degree > 3 || !opts_ok(opts)) return STEEPGS_ERR_INVALID_ARG;
  if (n == 0) return STEEPGS_OK;
  if (!d_params || !d_cams || !d_splats || !d_tiles_touched || !d_depth_keys) return STEEPGS_ERR_INVALID_ARG;
  if ((int64_t)V * n >= (int64_t)UINT32_MAX) return STEEPGS_ERR_INVALID_ARG;  // record ids are 32-bit
  timer_begin(STEEPGS_TIMER_PROJECT, as_stream(stream));
  const dim3 pg((unsigned)ceil_div(n, kProjThreads)), pb(kProjThreads);
  hipStream_t st = as_stream(stream);
  switch (sh_degree) {
    case 0: hipLaunchKernelGGL(k_project<0>, pg, pb, 0, st, d_params, n, d_cams, V, *opts, d_splats, d_tiles_touched, d_depth_keys); break;
    case 1: hipLaunchKernelGGL(k_project<1>, pg, pb, 0, st, d_params, n, d_cams, V, *opts, d_splats, d_tiles_touched, d_depth_keys); break;
    case 2: hipLaunchKernelGGL(k_project<2>, pg, pb, 0, st, d_params, n, d_cams, V, *opts, d_splats, d_tiles_touched, d_depth_keys); break;
    default: hipLaunchKernelGGL(k_project<3>, pg, pb, 0, st, d_params, n, d_cams, V, *opts, d_splats, d_tiles_touched, d_depth_keys); break;
  }
  timer_end(STEEPGS_TIMER_PROJECT, as_stream(stream));
  SG_TRY_LAUNCH();
  return STEEPGS_OK;
}

extern "C" steepgs_status steepgs_layout_cameras(steepgs_camera* cams, int32_t V, const steepgs_opts* opts,
                                                 int64_t* total_pixels, int32_t* total_tiles) {
  if (!cams || V <= 0 || !opts_ok(opts)) return STEEPGS_ERR_INVALID_ARG;
  int64_t poff = 0, toff = 0;
  for (int v = 0; v < V; ++v) {
    steepgs_camera& c = cams[v];
    if (c.width <= 0 || c.height <= 0 || c.width > 65535 * 8 || c.height > 65535 * 8) return STEEPGS_ERR_INVALID_ARG;
    if (c.model != 0 && c.model != 1) return STEEPGS_ERR_INVALID_ARG;
    c.tiles_x = (c.width + opts->tile_w - 1) / opts->tile_w;
    c.tiles_y = (c.height + opts->tile_h - 1) / opts->tile_h;
    c.tile_offset = (int32_t)toff;
    c.pixel_offset = poff;
    toff += (int64_t)c.tiles_x * c.tiles_y;
    poff += (int64_t)c.width * c.height;
    if (toff >= (int64_t)1 << 31) return STEEPGS_ERR_INVALID_ARG;
  }
  if (total_pixels) *total_pixels = poff;
  if (total_tiles) *total_tiles = (int32_t)toff;
  return STEEPGS_OK;
}

extern "C" const char* steepgs_status_string(int32_t status) {
  switch (status) {
    case STEEPGS_OK: return "ok";
    case STEEPGS_ERR_INVALID_ARG: return "invalid argument";
    case STEEPGS_ERR_CAPACITY: return "output capacity exceeded";
    case STEEPGS_ERR_HIP: return "HIP runtime error";
    case STEEPGS_ERR_WORKSPACE: return "workspace too small";
  }
  return "unknown status";
}

extern "C" const char* steepgs_version(void) { return "steepgs-gfx950 0.1"; }

namespace sg {
KernelTimer* kernel_timers() {
  static KernelTimer timers[STEEPGS_TIMER_COUNT];
  return timers;
}

int device_cu_count() {
  static int cache[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
  if (cache[dev] == 0) {
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) cus = 256;
    cache[dev] = cus;
  }
  return cache[dev];
}
}  // namespace sg

namespace sg {
size_t sort_workspace(int64_t m, uint64_t cap);
size_t render_fwd_workspace();
size_t render_bwd_workspace(int64_t m);
size_t densify_workspace(int64_t n);
size_t render_bwd6_workspace(int64_t m);
}  // namespace sg

extern "C" size_t steepgs_workspace_size(int32_t stage, int64_t n, int32_t V, uint64_t capacity,
                                         int32_t total_tiles) {
  (void)total_tiles;
  if (n < 0 || V < 0) return 0;
  const int64_t m = (int64_t)V * n;
  switch (stage) {
    case 1: return sg::sort_workspace(m, capacity);
    case 2: return sg::render_fwd_workspace();
    case 3: return sg::render_bwd_workspace(m);
    case 4: return sg::densify_workspace(n);
    case 5: return sg::render_bwd6_workspace(m);
    default: return 0;
  }
}

extern "C" steepgs_status steepgs_set_kernel_timer(int32_t which, void* const* start_events,
                                                   void* const* stop_events, int32_t count) {
  if (which < 0 || which >= STEEPGS_TIMER_COUNT || count < 0 || count > 1024) return STEEPGS_ERR_INVALID_ARG;
  if (count > 0 && (!start_events || !stop_events)) return STEEPGS_ERR_INVALID_ARG;
  sg::KernelTimer& t = sg::kernel_timers()[which];
  for (int i = 0; i < count; ++i) {
    t.starts[i] = reinterpret_cast<hipEvent_t>(start_events[i]);
    t.stops[i] = reinterpret_cast<hipEvent_t>(stop_events[i]);
  }
  t.count = count;
  t.next = 0;
  return STEEPGS_OK;
}
