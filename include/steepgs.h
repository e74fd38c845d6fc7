/*
 * steepgs.h -- C ABI of the SteepGS hot path on AMD Instinct MI355X (gfx950).
 *
 * Paper: "Steepest Descent Density Control for Compact 3D Gaussian
 * Splatting" (arXiv 2505.05587).  The five stages are
 *
 *   steepgs_project          Sec. 3, Eq. (sigma_3D), Eq. (sigma_2D) and the
 *                            footnote on Pi: each Gaussian through each camera.
 *   steepgs_sort             Sec. 3 "Rasterization": view-dependent depth order,
 *                            grouped by screen tile.
 *   steepgs_render_fwd       Sec. 3, Eq. (alpha_blend), front-to-back; Eq. (loss)
 *                            L1 value when a target is given.
 *   steepgs_render_bwd_split Sec. 4.4 and Theorem 1: backward of the blend and the
 *                            per-Gaussian splitting matrix
 *                            S_i += sum_x dL/dalpha_i(x) * Hessian_p alpha_i(x),
 *                            with the Hessian of Sec. 4.4 / App. C.4.
 *   steepgs_densify          Theorem 2, Algorithm 1, App. A.3: smallest
 *                            eigenpair of each 3x3 S_i, split iff
 *                            lambda_min < eps_split into p +/- eps v_min with
 *                            half the opacity each.
 *
 * General conventions
 *   - Every pointer named d_* is device memory owned by the caller.  The
 *     library never allocates, frees or keeps device memory between calls;
 *     scratch space comes from the caller's workspace (see
 *     steepgs_workspace_size; 4-byte alignment suffices, the library aligns
 *     its own sub-buffers).  Host pointers are read during the call only.
 *   - `stream` is a hipStream_t.  Calls only enqueue work on it: no host
 *     synchronisation, no device allocation and no memset nodes, so every call
 *     may be captured into a HIP graph.  Calls that overlap on one workspace
 *     race.
 *   - Return value: STEEPGS_OK, or an error detected on the host before any
 *     work is enqueued (bad argument, launch failure).  Failures that depend on
 *     data (instance or output capacity) are written to *d_status on the
 *     device together with the size that would have been needed.
 *   - Floating point is IEEE fp32 storage.  Projection, eigensolve and the
 *     geometric part of the projection backward (camera map, Pi(Sigma), its
 *     inverse, quaternion and scale, splitting-matrix lift) compute in fp64;
 *     the rasterizer and the SH colour in fp32.  The backward sums each
 *     Gaussian's per-tile float32 partials in fp64, so its results do not
 *     depend on the order in which the tiles finish: repeated launches on
 *     the same inputs give bit-identical gradients and S.
 *
 * Gaussian parameters: one planar float32 array [F][n] (row stride n),
 *   rows 0-2 position p, 3-5 log-scales, 6-9 quaternion (w,x,y,z) (normalised
 *   inside), 10 opacity logit, 11.. SH coefficients: row 11 + 3*k + channel,
 *   basis k = l*l + l + m of the real spherical harmonics (Condon-Shortley
 *   phase), F = 11 + 3*(d+1)^2 for SH degree d in 0..3.
 *   covariance = R(q) diag(exp(2*log_scale)) R(q)^T, opacity = sigmoid(logit),
 *   colour = max(0, sum_k sh_k Y_k(dir) + 1/2), dir = unit(p - camera centre).
 */
#ifndef STEEPGS_H
#define STEEPGS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  STEEPGS_OK = 0,
  STEEPGS_ERR_INVALID_ARG = 1, /* null pointer, bad size, unsupported option */
  STEEPGS_ERR_CAPACITY = 2,    /* (device status) an output buffer was too small */
  STEEPGS_ERR_HIP = 3,         /* a HIP launch or runtime call failed */
  STEEPGS_ERR_WORKSPACE = 4    /* workspace smaller than steepgs_workspace_size() */
} steepgs_status;

#define STEEPGS_ROW_MEAN 0
#define STEEPGS_ROW_LOG_SCALE 3
#define STEEPGS_ROW_QUAT 6
#define STEEPGS_ROW_OPACITY 10
#define STEEPGS_ROW_SH 11
#define STEEPGS_NUM_PARAMS(d) (11 + 3 * ((d) + 1) * ((d) + 1))

/* One camera (96 bytes).  World->camera x_c = R x + t, camera looks down +z,
 * x right, y down.  model 0 (pinhole): u = fx x_c/z_c + cx, v = fy y_c/z_c + cy;
 * model 1 (orthographic): u = fx x_c + cx, v = fy y_c + cy.  Pixel (u, v)
 * (integers) is sampled at the image point (u, v).  tiles_x, tiles_y,
 * tile_offset and pixel_offset place the view in the batch and are filled by
 * steepgs_layout_cameras. */
typedef struct {
  float R[9]; /* row-major */
  float t[3];
  float fx, fy, cx, cy;
  int32_t width, height;
  int32_t model;
  int32_t tiles_x, tiles_y;
  int32_t tile_offset;  /* global id of the view's first tile */
  int64_t pixel_offset; /* index of the view's first pixel in packed images */
} steepgs_camera;

/* Raster conventions (host struct, read at call time).  alpha_min = 0,
 * alpha_max = 1, t_min = 0 gives the cut-off free "smooth" blend; alpha is
 * capped at 1 - 2^-24 (the largest float below one) even then, so that
 * 1 - alpha never vanishes for a saturated opacity.
 *   alpha = min(alpha_max, o * exp(-1/2 d^T A d)); entries with alpha < alpha_min
 *   are skipped; a pixel stops before the entry that would take its
 *   transmittance below t_min.
 *   footprint radius = ceil(radius_sigmas * sqrt(lambda_max(Pi(Sigma)))) pixels;
 *   dilation is added to the diagonal of Pi(Sigma); frustum_guard > 0 clamps
 *   x_c/z_c, y_c/z_c to +/- frustum_guard * half-image-size / focal inside the
 *   pinhole Jacobian; Gaussians with z_c <= near_z are culled. */
typedef struct {
  int32_t tile_w, tile_h; /* supported: 16x16, 16x8, 8x8 */
  float near_z;
  float radius_sigmas;
  float dilation;
  float frustum_guard;
  float alpha_min, alpha_max, t_min;
  float bg[3];
  /* launch shape of the persistent raster kernels (results do not depend on
   * it): workgroups per compute unit (0: 8; 1..64) and wavefronts per
   * workgroup (0: 4; 2, 4 or 8), each wavefront working on a tile of its
   * own; chosen by the autotuner */
  int32_t raster_wgs_per_cu;
  int32_t raster_waves_per_wg;
} steepgs_opts;

/* Projected record of one (view, Gaussian) pair, 64 bytes.  Index r = v*n + i.
 * mean = the projected mean rounded to float32; mean_lo packs what that
 * rounding dropped, mean_x_exact - mean_x in the low 16 bits and
 * mean_y_exact - mean_y in the high 16 bits, each an IEEE binary16 (the
 * blend evaluates pixel offsets from the mean to ~2^-24 of the offset rather
 * than of the pixel coordinate).  The depth of a record is not stored here:
 * steepgs_project writes it to the depth-key array.
 * conic = (a, b, c) with A = [[a, b], [b, c]] = Pi(Sigma)^-1.  rect packs the
 * inclusive tile rectangle: rect_lo = x0 | y0 << 16, rect_hi = x1 | y1 << 16.
 * A pair is culled when tiles_touched is 0; a pair culled by the projection
 * itself (near plane, degenerate conic, empty rectangle) also has opacity 0.
 * The fields the footprint walk reads (mean, conic, opacity, rect) come first,
 * in one 32-byte block: the instance emission gathers records in depth order.
 * The last block is the conic in eigen form, from which the blend evaluates
 * alpha: (axis_x, axis_y) the unit long axis of the footprint ellipse,
 * e_long, e_short = -log2(e)/2 times the conic's eigenvalues along the long
 * and the short axis, so that -1/2 d^T A d = ln 2 * (e_long (axis . d)^2 +
 * e_short (axis_perp . d)^2), axis_perp = (-axis_y, axis_x).  (A sum of two
 * non-negative terms: in float32 its error grows with the square root of the
 * ellipse's aspect ratio, not with the aspect ratio as a, b, c's terms do.)
 * All computed in fp64 from Pi(Sigma) and rounded once. */
typedef struct {
  float mean_x, mean_y;
  float conic_a, conic_b;
  float conic_c, opacity;
  uint32_t rect_lo, rect_hi;
  float rgb[3];
  uint32_t mean_lo; /* binary16 remainders of the mean, x | y << 16 */
  float axis_x, axis_y;
  float e_long, e_short;
} steepgs_splat;

/* Fill tiles_x/tiles_y/tile_offset/pixel_offset of V host cameras for the
 * tile shape of `opts`; returns the totals.  Host only. */
steepgs_status steepgs_layout_cameras(steepgs_camera* cams, int32_t V, const steepgs_opts* opts,
                                      int64_t* total_pixels, int32_t* total_tiles);

/* Workspace (device bytes) each stage needs.  stage: 1 sort, 2 render_fwd,
 * 3 render_bwd_split, 4 densify (and densify6), 5 render_bwd_split6 (project
 * needs none).  n = Gaussians, V = views, capacity = instance capacity of the
 * sort. */
size_t steepgs_workspace_size(int32_t stage, int64_t n, int32_t V, uint64_t capacity, int32_t total_tiles);

/* Stage 1 -- projection (Sec. 3, Eqs. sigma_3D / sigma_2D).
 * In:  d_params [F][n], d_cams [V] (device copy of laid-out cameras).
 * Out: d_splats [V*n], d_tiles_touched [V*n]: the number of tiles of the
 *      record's tile rectangle (a bound of its instance count; the exact
 *      count is an output of steepgs_sort), 0 if culled.  Discrete outcomes
 *      (culling, rectangle, depth) are computed in fp64 in a fixed operation
 *      order.
 *      d_depth_keys [V*n]: the keys of steepgs_sort's depth order, the
 *      float bits of each record's camera-space depth (rounded once from
 *      fp64), 0xFFFFFFFF for a culled record (steepgs_sort takes them). */
steepgs_status steepgs_project(const float* d_params, int64_t n, int32_t sh_degree, const steepgs_camera* d_cams,
                               int32_t V, const steepgs_opts* opts, steepgs_splat* d_splats,
                               uint32_t* d_tiles_touched, uint32_t* d_depth_keys, void* stream);

/* Stage 2 -- instance list (Sec. 3 "Rasterization": sort by view-dependent
 * depth).  One instance per (record, tile of its rectangle whose box of pixel
 * centres meets the footprint ellipse d^T A d <= radius_sigmas^2; tested in
 * fp64 on the stored float32 mean and conic, 1e-6 relative slack); 64-bit
 * key global_tile << 32 | float bits of depth; value r = v*n + i; sorted by
 * key, ties by r (the order of emission view, Gaussian, row-major tile).
 * Out: d_vals [capacity] sorted values; d_keys [capacity] (nullable) sorted
 *      keys; d_tile_ranges [total_tiles][2] = [begin, end) ((0,0) if empty);
 *      d_counts [V*n] (nullable): each record's instance count (0 if culled);
 *      *d_num_instances = K.  If K > capacity, *d_status = STEEPGS_ERR_CAPACITY,
 *      *d_num_instances holds K and the outputs other than d_counts are not
 *      written.  *d_status is set to 0 otherwise.
 * d_tiles_touched [V*n]: as steepgs_project wrote it (0: culled).
 * d_depth_keys [V*n]: the depth keys steepgs_project wrote for these same
 *      records (required; read only). */
steepgs_status steepgs_sort(const steepgs_splat* d_splats, const uint32_t* d_tiles_touched,
                            const uint32_t* d_depth_keys, int64_t n, int32_t V,
                            const steepgs_camera* d_cams, const steepgs_opts* opts, int32_t total_tiles,
                            uint64_t* d_keys, uint32_t* d_vals, uint64_t capacity, uint32_t* d_tile_ranges,
                            uint32_t* d_counts, uint64_t* d_num_instances, int32_t* d_status, void* d_ws,
                            size_t ws_bytes, void* stream);

/* Stage 3 -- forward blend (Eq. alpha_blend), all V views in one persistent
 * launch.  Out: d_image packed per view as [3][H][W] planes (offset
 * 3*pixel_offset), d_T_final [total_pixels], d_n_contrib [total_pixels]
 * (entries of the tile list up to and including the last contributor).
 * d_n_used (nullable) [total_pixels]: number of entries blended into the pixel.
 * d_target (nullable, same layout as d_image): when given, d_loss[V] receives
 * the per-view mean absolute error of Eq. (loss) (overwritten). */
steepgs_status steepgs_render_fwd(const steepgs_splat* d_splats, int64_t n, const uint32_t* d_vals,
                                  const uint32_t* d_tile_ranges, const steepgs_camera* d_cams, int32_t V,
                                  const steepgs_opts* opts, int32_t total_tiles, int64_t total_pixels,
                                  const float* d_target, float* d_image, float* d_T_final, uint32_t* d_n_contrib,
                                  uint32_t* d_n_used, float* d_loss, void* d_ws, size_t ws_bytes, void* stream);

/* steepgs_render_fwd without a workspace argument, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same inputs, outputs, errors and results
 * as steepgs_render_fwd.  Its scratch -- the persistent launch's 4-byte
 * tile-queue counter, cleared by a kernel at every call -- lives in a
 * 256-byte file-scope device array of the library, one copy per GPU, which
 * the GPU holds until the process ends; its address is looked up on the
 * first call on each device (current device at call time, at most 64
 * devices; the stream must belong to that device).  The call allocates
 * nothing.  Every call on one GPU shares that array: calls that overlap on
 * one GPU (other streams, other host threads) race; calls in stream order
 * do not.  STEEPGS_ERR_WORKSPACE if the forward ever needed more scratch
 * than the array holds; STEEPGS_ERR_HIP if the array cannot be located. */
steepgs_status steepgs_render_fwd_noalloc(const steepgs_splat* d_splats, int64_t n, const uint32_t* d_vals,
                                          const uint32_t* d_tile_ranges, const steepgs_camera* d_cams, int32_t V,
                                          const steepgs_opts* opts, int32_t total_tiles, int64_t total_pixels,
                                          const float* d_target, float* d_image, float* d_T_final,
                                          uint32_t* d_n_contrib, uint32_t* d_n_used, float* d_loss, void* stream);

/* Stage 4 -- backward of the blend and the projection, and the splitting
 * matrices (Theorem 1; Sec. 4.4).  Loss gradient per pixel: d_dL_dimage when
 * non-null, else the L1 loss of Eq. (loss) against d_target (sum over views
 * of the per-view mean).  Accumulates (+=, caller zeroes):
 *   d_grads [F][n]  dL/dparams,
 *   d_S     [6][n]  S_i summed over views and pixels, entries xx xy xz yy yz zz,
 *                   with Hessian_p alpha = alpha P^T (A d d^T A - A) P, P the
 *                   Jacobian of the projected mean w.r.t. p, held fixed with
 *                   Pi(Sigma) and colour (App. C.4).
 * d_grad2d (nullable) [V*n][12] receives the per-pair gradients w.r.t.
 * (mean_x, mean_y, conic a, b, c, opacity, r, g, b) in entries 0-8 of each
 * 48-byte slot (overwritten; entries 9-11 and culled pairs are zero), rounded
 * from the fp64 sums in the workspace (steepgs_workspace_size(3, ...) bytes
 * are needed either way).
 * With n = 0 nothing is accumulated and the per-Gaussian buffers (params,
 * records, counts, grads, S) may be null. */
steepgs_status steepgs_render_bwd_split(const float* d_params, int64_t n, int32_t sh_degree,
                                        const steepgs_camera* d_cams, int32_t V, const steepgs_opts* opts,
                                        const steepgs_splat* d_splats, const uint32_t* d_tiles_touched,
                                        const uint32_t* d_vals, const uint32_t* d_tile_ranges, int32_t total_tiles,
                                        int64_t total_pixels, const float* d_image, const float* d_T_final,
                                        const uint32_t* d_n_contrib, const float* d_dL_dimage,
                                        const float* d_target, float* d_grads, float* d_S, float* d_grad2d,
                                        void* d_ws, size_t ws_bytes, void* stream);

/* The backward's first step, on its own: clears the fp64 moment slots of a
 * stage-3 workspace (steepgs_workspace_size(3, n, V, ...) bytes, laid out for
 * n and V), which steepgs_render_bwd_split accumulates into.  With
 * steepgs_render_bwd_split_cleared it lets a caller run the clear earlier,
 * on another stream -- e.g. beside the forward blend, which leaves most of
 * the HBM bandwidth unused.  The workspace is the caller's; n = 0 does
 * nothing.  STEEPGS_ERR_INVALID_ARG for n < 0, V <= 0 or a null workspace,
 * STEEPGS_ERR_WORKSPACE if ws_bytes is too small. */
steepgs_status steepgs_render_bwd_clear(int64_t n, int32_t V, void* d_ws, size_t ws_bytes, void* stream);

/* steepgs_render_bwd_split without its own clear of the workspace's moment
 * slots (same arguments, results and errors): the caller has cleared them
 * with steepgs_render_bwd_clear for the same n and V, ordered before this
 * call (same stream, or an event), and nothing else has written the
 * workspace since.  Slots left uncleared add into the results. */
steepgs_status steepgs_render_bwd_split_cleared(const float* d_params, int64_t n, int32_t sh_degree,
                                                const steepgs_camera* d_cams, int32_t V, const steepgs_opts* opts,
                                                const steepgs_splat* d_splats, const uint32_t* d_tiles_touched,
                                                const uint32_t* d_vals, const uint32_t* d_tile_ranges,
                                                int32_t total_tiles, int64_t total_pixels, const float* d_image,
                                                const float* d_T_final, const uint32_t* d_n_contrib,
                                                const float* d_dL_dimage, const float* d_target, float* d_grads,
                                                float* d_S, float* d_grad2d, void* d_ws, size_t ws_bytes,
                                                void* stream);

/* Stage 4 over theta = (p, log-scales) (dim 6; Sec. 4.4 defines S_i over the
 * parameters the Hessian is taken in, the paper's experiments use p alone):
 * as steepgs_render_bwd_split, and in addition
 *   d_S6 [21][n] (+=) the 6x6 splitting matrix, upper triangle row-major
 *                over (p_x, p_y, p_z, s_x, s_y, s_z) (s = log-scales):
 *                sum over views and contributing unclamped pixels of
 *                dL/dalpha * Hessian_theta alpha, with the projection's maps
 *                frozen at the point (the mean moves along the exact
 *                Jacobian of the projection, the 2D covariance is
 *                P Sigma(s) P^T + dilation with P at the guarded point;
 *                App. C.4's approximation, extended to the scales).
 * d_S (nullable here) receives the dim-3 S as before.  No d_grad2d output.
 * Workspace: steepgs_workspace_size(5, ...). */
steepgs_status steepgs_render_bwd_split6(const float* d_params, int64_t n, int32_t sh_degree,
                                         const steepgs_camera* d_cams, int32_t V, const steepgs_opts* opts,
                                         const steepgs_splat* d_splats, const uint32_t* d_tiles_touched,
                                         const uint32_t* d_vals, const uint32_t* d_tile_ranges, int32_t total_tiles,
                                         int64_t total_pixels, const float* d_image, const float* d_T_final,
                                         const uint32_t* d_n_contrib, const float* d_dL_dimage,
                                         const float* d_target, float* d_grads, float* d_S, float* d_S6,
                                         void* d_ws, size_t ws_bytes, void* stream);

/* Optional selection rules of the split step (the paper's "Variants" and
 * Algorithm 1's "condition on G"):
 *  - compactest splitting: a Gaussian is a candidate only when also
 *    |g_scale * G_i| <= eps_grad, G = d_G [3][n] the accumulated gradient of
 *    the position (Algorithm 1's G; g_scale = 1 / T_split averages it); the
 *    norm is compared squared in fp64.  d_G = NULL or eps_grad <= 0: off.
 *  - ADC-style gate (the condition of the adaptive density control that the
 *    "Variants" section contrasts with the compactest rule, on the mean of
 *    the gradient's norm rather than the norm of its mean): a candidate only
 *    when also g_scale * Gabs_i >= adc_tau, Gabs = d_Gabs [n] the
 *    accumulated per-step norm of the position gradient (steepgs_adam_step
 *    accumulates it); compared in fp64.  d_Gabs = NULL or adc_tau <= 0: off.
 *  - increment budget: when more than `budget` Gaussians are candidates,
 *    only the `budget` ones with the smallest lambda_min split (ties: lower
 *    index first), compared on the float32 lambda_min the call reports.
 *    budget <= 0: no limit. */
typedef struct {
  const float* d_G;
  float g_scale;
  float eps_grad;
  int64_t budget;
  const float* d_Gabs;
  float adc_tau;
} steepgs_split_select;

/* Stage 5 -- Steepest Density Control (Theorem 2; Algorithm 1; App. A.3).
 * S' = s_scale * S (Algorithm 1 averages over the interval); smallest
 * eigenpair by the trigonometric root formula in fp64; split iff
 * lambda_min < eps_split, and the rules of `select` (host pointer, nullable:
 * none).  Output layout: exclusive scan of m_i in {1, 2}:
 * d_out [F][out_capacity] row stride out_capacity; an unsplit Gaussian is
 * copied to out[off_i]; a split one writes (p + eps v_min, o/2) to off_i and
 * (p - eps v_min, o/2) to off_i + 1 (opacity halved in [0,1], logit re-derived;
 * other rows copied).  *d_n_out = n + #splits.  d_lambda_min [n], d_vmin [3][n]
 * (unit, largest-magnitude component positive), d_split [n] (nullable each).
 * If n + #splits > out_capacity: *d_status = STEEPGS_ERR_CAPACITY, *d_n_out holds
 * the needed size and d_out is not written. */
steepgs_status steepgs_densify(const float* d_params, int64_t n, int32_t sh_degree, const float* d_S, float s_scale,
                               float eps, float eps_split, const steepgs_split_select* select, float* d_out,
                               int64_t out_capacity, int64_t* d_n_out,
                               float* d_lambda_min, float* d_vmin, uint8_t* d_split, int32_t* d_status, void* d_ws,
                               size_t ws_bytes, void* stream);

/* Stage 5 over theta = (p, log-scales): S' = s_scale * S6 (d_S6 [21][n] as
 * steepgs_render_bwd_split6 fills it); smallest eigenpair of the 6x6 by cyclic
 * Jacobi rotations in fp64; split iff lambda_min < eps_split; the offspring
 * move by +- eps v_min in theta -- position rows 0-2 and log-scale rows 3-5
 * -- and take o/2 (logit re-derived); other rows copied.  Layout, capacity,
 * status and outputs as steepgs_densify, with d_vmin [6][n].  Workspace:
 * steepgs_workspace_size(4, ...). */
steepgs_status steepgs_densify6(const float* d_params, int64_t n, int32_t sh_degree, const float* d_S6,
                                float s_scale, float eps, float eps_split, float* d_out, int64_t out_capacity,
                                int64_t* d_n_out, float* d_lambda_min, float* d_vmin, uint8_t* d_split,
                                int32_t* d_status, void* d_ws, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------------------
 * Training-loop support (Algorithm 1 around the hot path). */

/* Adam hyper-parameters; lr per parameter group: position, log-scales,
 * quaternion, opacity logit, SH degree 0, SH degrees >= 1. */
typedef struct {
  float lr[6];
  float beta1, beta2, eps;
} steepgs_adam_opts;

/* One Adam step, the optimizer of the 3DGS training pipeline that Sec. 5.1
 * keeps: t = ++*d_step (device int64), m = b1 m + (1 - b1) g,
 * v = b2 v + (1 - b2) g^2, p -= (lr / (1 - b1^t)) m / (sqrt(v) / sqrt(1 - b2^t)
 * + eps) elementwise over d_params, d_grads, d_m, d_v [F][n] (fp32; the bias
 * corrections in fp64).  d_G [3][n] (nullable) accumulates the position
 * gradient (Algorithm 1's G += grad); d_Gabs [n] (nullable) accumulates its
 * Euclidean norm (fp32), the statistic of the ADC-style gate.  Errors:
 * INVALID_ARG for a null pointer, a degree outside 0..3, betas outside
 * [0, 1) or eps <= 0. */
steepgs_status steepgs_adam_step(float* d_params, const float* d_grads, float* d_m, float* d_v, int64_t n,
                                 int32_t sh_degree, const steepgs_adam_opts* opts, int64_t* d_step, float* d_G,
                                 float* d_Gabs, void* stream);

/* Per-Gaussian state (e.g. Adam moments) onto the layout of a densification
 * (Algorithm 1's replacement of a split Gaussian by two offspring): with
 * d_split [n] the flags steepgs_densify reported, a kept Gaussian i's rows
 * d_src[r][i] (rows x n) go to d_dst[r][i + #splits before i] (row stride
 * dst_capacity), and both offspring slots of a split one are zero (fresh
 * state).  Slots at or beyond dst_capacity are not written.  Workspace: at
 * least steepgs_workspace_size(4, n, 1, 0, 0) bytes. */
steepgs_status steepgs_split_remap(const float* d_src, int32_t rows, int64_t n, const uint8_t* d_split, float* d_dst,
                                   int64_t dst_capacity, void* d_ws, size_t ws_bytes, void* stream);

/* Profiling hook.  When set for kernel `which` (STEEPGS_TIMER_*), every
 * later launch of that kernel records start_events[i] immediately before and
 * stop_events[i] immediately after it on the launch's stream, i = 0, 1, ...
 * cycling through `count` caller-owned hipEvent_t handles, so a caller can time
 * a kernel live inside a run.  count = 0 clears it.  Host-side process-global
 * setting; not thread-safe; never allocates. */
#define STEEPGS_TIMER_PROJECT 0    /* projection kernel */
#define STEEPGS_TIMER_SORT 1       /* whole instance-sort stage */
#define STEEPGS_TIMER_RENDER_FWD 2 /* forward raster kernel */
#define STEEPGS_TIMER_RENDER_BWD 3 /* backward raster kernel */
#define STEEPGS_TIMER_PROJ_BWD 4   /* projection backward + splitting-matrix lift */
#define STEEPGS_TIMER_DENSIFY 5    /* whole densification stage */
#define STEEPGS_TIMER_COUNT 6
steepgs_status steepgs_set_kernel_timer(int32_t which, void* const* start_events, void* const* stop_events,
                                        int32_t count);

/* Measurement support: the achievable fp32 vector-ALU rate.  Launches
 * `blocks` workgroups of 256 threads; every thread runs 8 independent fp32
 * fused multiply-add chains for `iters` steps (plain, not packed, FMA: the
 * instruction mix of the library's kernels) and writes one float to
 * d_out[blocks * 256].  flops = blocks * 256 * iters * 16.  Errors:
 * INVALID_ARG for a null d_out or a non-positive size. */
steepgs_status steepgs_calibrate_valu(float* d_out, int32_t blocks, int32_t iters, void* stream);

/* A static string naming status code `status` (any value: codes outside
 * steepgs_status give "unknown status"). */
const char* steepgs_status_string(int32_t status);
const char* steepgs_version(void);

#ifdef __cplusplus
}
#endif

#endif /* STEEPGS_H */
