"""ctypes binding of ``libsteepgs.so`` (the C ABI in ``include/steepgs.h``).

Argument marshalling only: every entry point here has the name of the C
function it calls, takes torch tensors that live on the GPU, passes their
device pointers and the current HIP stream, and raises on a non-OK status.
No computation happens in Python.
"""
from __future__ import annotations

import ctypes as C
import os

import torch  # loads the HIP runtime the library binds to

_HERE = os.path.dirname(os.path.abspath(__file__))
# STEEPGS_LIB: another build of the same library (A/B timing of build variants)
LIB_PATH = os.environ.get("STEEPGS_LIB") or os.path.join(_HERE, "libsteepgs.so")

STATUS = {0: "ok", 1: "invalid argument", 2: "output capacity exceeded", 3: "HIP runtime error",
          4: "workspace too small"}
OK, ERR_INVALID_ARG, ERR_CAPACITY, ERR_HIP, ERR_WORKSPACE = 0, 1, 2, 3, 4
STAGE_SORT, STAGE_RENDER_FWD, STAGE_RENDER_BWD, STAGE_DENSIFY, STAGE_RENDER_BWD6 = 1, 2, 3, 4, 5


class Camera(C.Structure):
    _fields_ = [("R", C.c_float * 9), ("t", C.c_float * 3), ("fx", C.c_float), ("fy", C.c_float),
                ("cx", C.c_float), ("cy", C.c_float), ("width", C.c_int32), ("height", C.c_int32),
                ("model", C.c_int32), ("tiles_x", C.c_int32), ("tiles_y", C.c_int32),
                ("tile_offset", C.c_int32), ("pixel_offset", C.c_int64)]


class Opts(C.Structure):
    _fields_ = [("tile_w", C.c_int32), ("tile_h", C.c_int32), ("near_z", C.c_float),
                ("radius_sigmas", C.c_float), ("dilation", C.c_float), ("frustum_guard", C.c_float),
                ("alpha_min", C.c_float), ("alpha_max", C.c_float), ("t_min", C.c_float),
                ("bg", C.c_float * 3), ("raster_wgs_per_cu", C.c_int32), ("raster_waves_per_wg", C.c_int32)]


class SplitSelect(C.Structure):
    _fields_ = [("d_G", C.c_void_p), ("g_scale", C.c_float), ("eps_grad", C.c_float), ("budget", C.c_int64),
                ("d_Gabs", C.c_void_p), ("adc_tau", C.c_float)]


class AdamOpts(C.Structure):
    _fields_ = [("lr", C.c_float * 6), ("beta1", C.c_float), ("beta2", C.c_float), ("eps", C.c_float)]


assert C.sizeof(Camera) == 96
SPLAT_FLOATS = 16  # 64-byte record


class SteepGSError(RuntimeError):
    def __init__(self, fn, status):
        super().__init__(f"{fn} failed: {STATUS.get(status, status)}")
        self.status = status


_lib = None


def lib():
    """Load the HIP library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_2505_05587_amd.build.build_library()")
        L = C.CDLL(LIB_PATH)
        vp, i64, i32, u64, f32, sz = C.c_void_p, C.c_int64, C.c_int32, C.c_uint64, C.c_float, C.c_size_t
        L.steepgs_layout_cameras.argtypes = [C.POINTER(Camera), i32, C.POINTER(Opts), C.POINTER(C.c_int64),
                                             C.POINTER(C.c_int32)]
        L.steepgs_workspace_size.argtypes = [i32, i64, i32, u64, i32]
        L.steepgs_workspace_size.restype = sz
        L.steepgs_project.argtypes = [vp, i64, i32, vp, i32, C.POINTER(Opts), vp, vp, vp, vp]
        L.steepgs_sort.argtypes = [vp, vp, vp, i64, i32, vp, C.POINTER(Opts), i32, vp, vp, u64, vp, vp, vp, vp, vp, sz,
                                   vp]
        L.steepgs_render_fwd.argtypes = [vp, i64, vp, vp, vp, i32, C.POINTER(Opts), i32, i64, vp, vp, vp, vp, vp,
                                         vp, vp, sz, vp]
        L.steepgs_render_fwd_noalloc.argtypes = [vp, i64, vp, vp, vp, i32, C.POINTER(Opts), i32, i64, vp, vp, vp,
                                                 vp, vp, vp, vp]
        L.steepgs_calibrate_valu.argtypes = [vp, i32, i32, vp]
        L.steepgs_calibrate_valu.restype = C.c_int
        L.steepgs_set_kernel_timer.argtypes = [i32, vp, vp, i32]
        L.steepgs_set_kernel_timer.restype = C.c_int
        L.steepgs_render_bwd_split.argtypes = [vp, i64, i32, vp, i32, C.POINTER(Opts), vp, vp, vp, vp, i32, i64,
                                               vp, vp, vp, vp, vp, vp, vp, vp, vp, sz, vp]
        L.steepgs_densify.argtypes = [vp, i64, i32, vp, f32, f32, f32, C.POINTER(SplitSelect), vp, i64, vp, vp, vp,
                                      vp, vp, vp, sz, vp]
        L.steepgs_render_bwd_split6.argtypes = L.steepgs_render_bwd_split.argtypes
        L.steepgs_render_bwd_split_cleared.argtypes = L.steepgs_render_bwd_split.argtypes
        L.steepgs_render_bwd_clear.argtypes = [i64, i32, vp, sz, vp]
        L.steepgs_densify6.argtypes = [vp, i64, i32, vp, f32, f32, f32, vp, i64, vp, vp, vp, vp, vp, vp, sz, vp]
        L.steepgs_adam_step.argtypes = [vp, vp, vp, vp, i64, i32, C.POINTER(AdamOpts), vp, vp, vp, vp]
        L.steepgs_split_remap.argtypes = [vp, i32, i64, vp, vp, i64, vp, sz, vp]
        for fn in ("steepgs_layout_cameras", "steepgs_project", "steepgs_sort", "steepgs_render_fwd",
                   "steepgs_render_fwd_noalloc",
                   "steepgs_render_bwd_split", "steepgs_densify", "steepgs_adam_step", "steepgs_split_remap",
                   "steepgs_render_bwd_split6", "steepgs_densify6", "steepgs_render_bwd_split_cleared",
                   "steepgs_render_bwd_clear"):
            getattr(L, fn).restype = C.c_int
        L.steepgs_status_string.argtypes = [C.c_int]
        L.steepgs_status_string.restype = C.c_char_p
        L.steepgs_version.restype = C.c_char_p
        _lib = L
    return _lib


def _p(t):
    """Device pointer of a tensor (or None)."""
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("expected a GPU tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return C.c_void_p(t.data_ptr())


def _stream(stream):
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _check(fn, st):
    if st != OK:
        raise SteepGSError(fn, st)


def make_opts(d: dict) -> Opts:
    o = Opts()
    o.tile_w, o.tile_h = int(d["tile_w"]), int(d["tile_h"])
    o.near_z, o.radius_sigmas, o.dilation = d["near_z"], d["radius_sigmas"], d["dilation"]
    o.frustum_guard, o.alpha_min, o.alpha_max, o.t_min = d["frustum_guard"], d["alpha_min"], d["alpha_max"], d["t_min"]
    for k in range(3):
        o.bg[k] = d["bg"][k]
    o.raster_wgs_per_cu = int(d.get("raster_wgs_per_cu", 0))
    o.raster_waves_per_wg = int(d.get("raster_waves_per_wg", 0))
    return o


def steepgs_layout_cameras(cams_arr, opts: Opts):
    """Fill the layout fields of a ctypes Camera array; returns (total_pixels, total_tiles)."""
    tp, tt = C.c_int64(0), C.c_int32(0)
    _check("steepgs_layout_cameras",
           lib().steepgs_layout_cameras(cams_arr, len(cams_arr), C.byref(opts), C.byref(tp), C.byref(tt)))
    return tp.value, tt.value


def steepgs_workspace_size(stage, n, V, capacity=0, total_tiles=0) -> int:
    return int(lib().steepgs_workspace_size(stage, n, V, capacity, total_tiles))


def steepgs_project(params, n, sh_degree, d_cams, V, opts, splats, tiles_touched, stream=None, depth_keys=None):
    _check("steepgs_project", lib().steepgs_project(_p(params), n, sh_degree, _p(d_cams), V, C.byref(opts),
                                                    _p(splats), _p(tiles_touched), _p(depth_keys), _stream(stream)))


def steepgs_sort(splats, tiles_touched, n, V, d_cams, opts, total_tiles, keys, vals, capacity, tile_ranges,
                 num_instances, status, ws, stream=None, depth_keys=None, counts=None):
    _check("steepgs_sort", lib().steepgs_sort(_p(splats), _p(tiles_touched), _p(depth_keys), n, V, _p(d_cams),
                                              C.byref(opts),
                                              total_tiles, _p(keys), _p(vals), capacity, _p(tile_ranges),
                                              _p(counts), _p(num_instances), _p(status), _p(ws), ws.numel() * ws.element_size(),
                                              _stream(stream)))


def steepgs_render_fwd(splats, n, vals, tile_ranges, d_cams, V, opts, total_tiles, total_pixels, target, image,
                       T_final, n_contrib, n_used, loss, ws, stream=None):
    _check("steepgs_render_fwd",
           lib().steepgs_render_fwd(_p(splats), n, _p(vals), _p(tile_ranges), _p(d_cams), V, C.byref(opts),
                                    total_tiles, total_pixels, _p(target), _p(image), _p(T_final), _p(n_contrib),
                                    _p(n_used), _p(loss), _p(ws), ws.numel() * ws.element_size(),
                                    _stream(stream)))


def steepgs_render_fwd_noalloc(splats, n, vals, tile_ranges, d_cams, V, opts, total_tiles, total_pixels, target,
                               image, T_final, n_contrib, n_used, loss, stream=None):
    _check("steepgs_render_fwd_noalloc",
           lib().steepgs_render_fwd_noalloc(_p(splats), n, _p(vals), _p(tile_ranges), _p(d_cams), V, C.byref(opts),
                                            total_tiles, total_pixels, _p(target), _p(image), _p(T_final),
                                            _p(n_contrib), _p(n_used), _p(loss), _stream(stream)))


def steepgs_calibrate_valu(out, blocks, iters, stream=None):
    _check("steepgs_calibrate_valu", lib().steepgs_calibrate_valu(_p(out), blocks, iters, _stream(stream)))


TIMER_PROJECT, TIMER_SORT, TIMER_RENDER_FWD, TIMER_RENDER_BWD, TIMER_PROJ_BWD, TIMER_DENSIFY = range(6)
TIMER_NAMES = ["project", "sort", "render_fwd", "render_bwd", "proj_bwd", "densify"]


def steepgs_set_kernel_timer(which, start_events, stop_events):
    """start_events / stop_events: lists of torch.cuda.Event (already created)
    or raw hipEvent_t handles; empty lists clear the timer."""
    def handle(e):
        return e.cuda_event if hasattr(e, "cuda_event") else int(e)
    cnt = len(start_events)
    arr_s = (C.c_void_p * max(cnt, 1))(*[handle(e) for e in start_events])
    arr_e = (C.c_void_p * max(cnt, 1))(*[handle(e) for e in stop_events])
    _check("steepgs_set_kernel_timer", lib().steepgs_set_kernel_timer(which, arr_s, arr_e, cnt))


def steepgs_render_bwd_split(params, n, sh_degree, d_cams, V, opts, splats, tiles_touched, vals, tile_ranges,
                             total_tiles, total_pixels, image, T_final, n_contrib, dL_dimage, target, grads, S,
                             grad2d, ws, stream=None):
    _check("steepgs_render_bwd_split",
           lib().steepgs_render_bwd_split(_p(params), n, sh_degree, _p(d_cams), V, C.byref(opts), _p(splats),
                                          _p(tiles_touched), _p(vals), _p(tile_ranges), total_tiles, total_pixels,
                                          _p(image), _p(T_final), _p(n_contrib), _p(dL_dimage), _p(target),
                                          _p(grads), _p(S), _p(grad2d), _p(ws), ws.numel() * ws.element_size(),
                                          _stream(stream)))


def steepgs_render_bwd_split_cleared(params, n, sh_degree, d_cams, V, opts, splats, tiles_touched, vals, tile_ranges,
                                     total_tiles, total_pixels, image, T_final, n_contrib, dL_dimage, target, grads,
                                     S, grad2d, ws, stream=None):
    """steepgs_render_bwd_split on a workspace cleared by steepgs_render_bwd_clear."""
    _check("steepgs_render_bwd_split_cleared",
           lib().steepgs_render_bwd_split_cleared(_p(params), n, sh_degree, _p(d_cams), V, C.byref(opts), _p(splats),
                                                  _p(tiles_touched), _p(vals), _p(tile_ranges), total_tiles,
                                                  total_pixels, _p(image), _p(T_final), _p(n_contrib),
                                                  _p(dL_dimage), _p(target), _p(grads), _p(S), _p(grad2d), _p(ws),
                                                  ws.numel() * ws.element_size(), _stream(stream)))


def steepgs_render_bwd_clear(n, V, ws, stream=None):
    _check("steepgs_render_bwd_clear",
           lib().steepgs_render_bwd_clear(n, V, _p(ws), ws.numel() * ws.element_size(), _stream(stream)))


def steepgs_render_bwd_split6(params, n, sh_degree, d_cams, V, opts, splats, tiles_touched, vals, tile_ranges,
                              total_tiles, total_pixels, image, T_final, n_contrib, dL_dimage, target, grads, S, S6,
                              ws, stream=None):
    _check("steepgs_render_bwd_split6",
           lib().steepgs_render_bwd_split6(_p(params), n, sh_degree, _p(d_cams), V, C.byref(opts), _p(splats),
                                           _p(tiles_touched), _p(vals), _p(tile_ranges), total_tiles, total_pixels,
                                           _p(image), _p(T_final), _p(n_contrib), _p(dL_dimage), _p(target),
                                           _p(grads), _p(S), _p(S6), _p(ws), ws.numel() * ws.element_size(),
                                           _stream(stream)))


def steepgs_densify6(params, n, sh_degree, S6, s_scale, eps, eps_split, out, out_capacity, n_out, lambda_min, vmin,
                     split, status, ws, stream=None):
    _check("steepgs_densify6",
           lib().steepgs_densify6(_p(params), n, sh_degree, _p(S6), float(s_scale), float(eps), float(eps_split),
                                  _p(out), out_capacity, _p(n_out), _p(lambda_min), _p(vmin), _p(split), _p(status),
                                  _p(ws), ws.numel() * ws.element_size(), _stream(stream)))


def steepgs_densify(params, n, sh_degree, S, s_scale, eps, eps_split, out, out_capacity, n_out, lambda_min, vmin,
                    split, status, ws, stream=None, G=None, g_scale=1.0, eps_grad=0.0, budget=0, Gabs=None,
                    adc_tau=0.0):
    """``G`` [3, n] / ``g_scale`` / ``eps_grad``: the compactest gate;
    ``Gabs`` [n] / ``adc_tau``: the ADC-style gate; ``budget``: the increment
    budget (all off by default)."""
    sel = None
    if G is not None or Gabs is not None or budget > 0:
        sel = SplitSelect(_p(G), float(g_scale), float(eps_grad), int(budget), _p(Gabs), float(adc_tau))
    _check("steepgs_densify",
           lib().steepgs_densify(_p(params), n, sh_degree, _p(S), float(s_scale), float(eps), float(eps_split),
                                 None if sel is None else C.byref(sel), _p(out), out_capacity, _p(n_out),
                                 _p(lambda_min), _p(vmin), _p(split), _p(status), _p(ws),
                                 ws.numel() * ws.element_size(), _stream(stream)))


def make_adam_opts(lr, beta1=0.9, beta2=0.999, eps=1e-15):
    """lr: six learning rates (position, log-scales, quaternion, opacity logit,
    SH degree 0, SH degrees >= 1)."""
    lr = list(lr)
    if len(lr) != 6:
        raise ValueError("six learning rates expected")
    return AdamOpts((C.c_float * 6)(*[float(x) for x in lr]), float(beta1), float(beta2), float(eps))


def steepgs_adam_step(params, grads, m, v, n, sh_degree, opts, step, G=None, Gabs=None, stream=None):
    _check("steepgs_adam_step",
           lib().steepgs_adam_step(_p(params), _p(grads), _p(m), _p(v), n, sh_degree, C.byref(opts), _p(step),
                                   _p(G), _p(Gabs), _stream(stream)))


def steepgs_split_remap(src, rows, n, split, dst, dst_capacity, ws, stream=None):
    _check("steepgs_split_remap",
           lib().steepgs_split_remap(_p(src), rows, n, _p(split), _p(dst), dst_capacity, _p(ws),
                                     ws.numel() * ws.element_size(), _stream(stream)))


def version() -> str:
    return lib().steepgs_version().decode()
