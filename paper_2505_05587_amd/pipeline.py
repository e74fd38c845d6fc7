"""Buffers and stage orchestration over the C ABI.

torch provides device memory and the stream; every stage runs in the HIP
library (``_lib``).  Nothing here computes.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

import numpy as np
import torch

from . import _lib as L


def _dev():
    if not torch.cuda.is_available():
        raise RuntimeError("the SteepGS HIP path needs a GPU")
    return torch.device("cuda", torch.cuda.current_device())


class CameraBatch:
    """V cameras laid out for one batched launch (device array of
    ``steepgs_camera``)."""

    def __init__(self, cams, opts: dict, device=None):
        self.opts_dict = dict(opts)
        self.opts = L.make_opts(opts)
        V = cams.V
        arr = (L.Camera * V)()
        for v in range(V):
            c = arr[v]
            R = np.asarray(cams.R[v], np.float32).reshape(9)
            for k in range(9):
                c.R[k] = float(R[k])
            for k in range(3):
                c.t[k] = float(cams.t[v][k])
            c.fx, c.fy, c.cx, c.cy = float(cams.fx[v]), float(cams.fy[v]), float(cams.cx[v]), float(cams.cy[v])
            c.width, c.height, c.model = int(cams.width[v]), int(cams.height[v]), int(cams.model[v])
        self.total_pixels, self.total_tiles = L.steepgs_layout_cameras(arr, self.opts)
        self.host = arr
        self.V = V
        self.widths = [int(w) for w in cams.width]
        self.heights = [int(h) for h in cams.height]
        self.pixel_offsets = [int(arr[v].pixel_offset) for v in range(V)]
        self.tile_offsets = [int(arr[v].tile_offset) for v in range(V)]
        raw = np.frombuffer(bytes(arr), dtype=np.uint8).copy()
        self.dev = torch.from_numpy(raw).to(device or _dev())

    def view_image(self, packed: torch.Tensor, v: int) -> torch.Tensor:
        o = 3 * self.pixel_offsets[v]
        h, w = self.heights[v], self.widths[v]
        return packed[o: o + 3 * h * w].view(3, h, w)


def _grow(t, numel, dtype, device):
    if t is None or t.numel() < numel:
        return torch.empty(max(int(numel), 1), dtype=dtype, device=device)
    return t


@dataclass
class ForwardState:
    K: int
    image: torch.Tensor
    T_final: torch.Tensor
    n_contrib: torch.Tensor
    loss: torch.Tensor | None


class Rasterizer:
    """Project, sort and blend a Gaussian set for a camera batch, and run the
    backward with splitting-matrix accumulation.  Buffers are kept and
    reused between calls."""

    def __init__(self, cams: CameraBatch, sh_degree: int, capacity: int = 0):
        self.cams = cams
        self.sh_degree = sh_degree
        self.dev = cams.dev.device
        self.capacity = int(capacity)
        self.n = -1
        self.splats = self.tiles = self.vals = self.keys = self.counts = None
        self.ranges = torch.empty(2 * cams.total_tiles, dtype=torch.int32, device=self.dev)
        self.num = torch.zeros(1, dtype=torch.int64, device=self.dev)
        self.status = torch.zeros(1, dtype=torch.int32, device=self.dev)
        self.ws_sort = self.ws_bwd = self.ws_bwd6 = None
        self.ws_fwd = torch.zeros(L.steepgs_workspace_size(L.STAGE_RENDER_FWD, 0, 1) // 4 + 64, dtype=torch.int32,
                                  device=self.dev)
        Px = cams.total_pixels
        self.image = torch.empty(3 * Px, dtype=torch.float32, device=self.dev)
        self.T_final = torch.empty(Px, dtype=torch.float32, device=self.dev)
        self.n_contrib = torch.empty(Px, dtype=torch.int32, device=self.dev)
        self.n_used = None
        self.loss = torch.zeros(cams.V, dtype=torch.float32, device=self.dev)
        self.grad2d = None

    # -- buffers ------------------------------------------------------------
    def _ensure(self, n: int, capacity: int):
        V = self.cams.V
        if n != self.n:
            self.splats = torch.empty((max(V * n, 1), L.SPLAT_FLOATS), dtype=torch.float32, device=self.dev)
            self.tiles = torch.empty(max(V * n, 1), dtype=torch.int32, device=self.dev)
            self.dkeys = torch.empty(max(V * n, 1), dtype=torch.int32, device=self.dev)
            self.ws_bwd = torch.empty(L.steepgs_workspace_size(L.STAGE_RENDER_BWD, n, V) // 4 + 64,
                                      dtype=torch.int32, device=self.dev)
            self.n = n
            self.ws_sort = None
        if capacity > self.capacity or self.vals is None or self.ws_sort is None:
            self.capacity = max(capacity, self.capacity, 1)
            self.vals = torch.empty(self.capacity, dtype=torch.int32, device=self.dev)
            self.ws_sort = torch.empty(
                L.steepgs_workspace_size(L.STAGE_SORT, n, V, self.capacity, self.cams.total_tiles) // 4 + 64,
                dtype=torch.int32,
                device=self.dev)

    # -- stages -------------------------------------------------------------
    def project(self, params: torch.Tensor):
        n = params.shape[1]
        self._ensure(n, self.capacity)
        L.steepgs_project(params, n, self.sh_degree, self.cams.dev, self.cams.V, self.cams.opts, self.splats,
                          self.tiles, depth_keys=self.dkeys)

    def sort(self, want_keys: bool = False, want_counts: bool = False) -> int:
        """Instance list; grows the capacity and retries on overflow (reads
        the instance count back to the host).  want_counts: each record's
        exact instance count into ``self.counts``."""
        n, V = self.n, self.cams.V
        counts = None
        if want_counts:
            self.counts = _grow(self.counts, max(V * n, 1), torch.int32, self.dev)
            counts = self.counts
        for _ in range(3):
            keys = None
            if want_keys:
                self.keys = _grow(self.keys, self.capacity, torch.int64, self.dev)
                keys = self.keys
            L.steepgs_sort(self.splats, self.tiles, n, V, self.cams.dev, self.cams.opts, self.cams.total_tiles, keys,
                           self.vals, self.capacity, self.ranges, self.num, self.status, self.ws_sort,
                           depth_keys=self.dkeys, counts=counts)
            K = int(self.num.item())
            if int(self.status.item()) == L.OK:
                return K
            self._ensure(n, int(K * 1.25) + 1024)
        raise RuntimeError("instance capacity could not be satisfied")

    def render(self, target: torch.Tensor | None = None, count_used: bool = False):
        if count_used and self.n_used is None:
            self.n_used = torch.empty(self.cams.total_pixels, dtype=torch.int32, device=self.dev)
        L.steepgs_render_fwd(self.splats, self.n, self.vals, self.ranges, self.cams.dev, self.cams.V, self.cams.opts,
                             self.cams.total_tiles, self.cams.total_pixels, target, self.image, self.T_final,
                             self.n_contrib, self.n_used if count_used else None,
                             self.loss if target is not None else None, self.ws_fwd)

    def forward(self, params: torch.Tensor, target: torch.Tensor | None = None, want_keys=False,
                count_used=False, want_counts=False) -> ForwardState:
        self.project(params)
        K = self.sort(want_keys, want_counts)
        self.render(target, count_used)
        return ForwardState(K, self.image, self.T_final, self.n_contrib, self.loss if target is not None else None)

    def clear_backward(self):
        """Clear the backward's moment slots ahead of ``backward(cleared=True)``
        (on the current stream, which may differ from the backward's)."""
        L.steepgs_render_bwd_clear(self.n, self.cams.V, self.ws_bwd)

    def backward(self, params: torch.Tensor, grads: torch.Tensor, S: torch.Tensor, target=None, dL_dimage=None,
                 keep_grad2d=False, cleared=False):
        """grads [F, n] and S [6, n] accumulate (+=).  cleared: the slots were
        cleared by ``clear_backward`` (ordered before this call)."""
        g2d = None
        if keep_grad2d:
            self.grad2d = _grow(self.grad2d, 12 * self.cams.V * self.n, torch.float32, self.dev)
            g2d = self.grad2d
        fn = L.steepgs_render_bwd_split_cleared if cleared else L.steepgs_render_bwd_split
        fn(params, self.n, self.sh_degree, self.cams.dev, self.cams.V, self.cams.opts, self.splats, self.tiles,
           self.vals, self.ranges, self.cams.total_tiles, self.cams.total_pixels, self.image, self.T_final,
           self.n_contrib, dL_dimage, target, grads, S, g2d, self.ws_bwd)

    def backward6(self, params: torch.Tensor, grads: torch.Tensor, S6: torch.Tensor, S: torch.Tensor | None = None,
                  target=None, dL_dimage=None):
        """As backward, and the splitting matrix over theta = (p, log-scales):
        S6 [21, n] (upper triangle of the 6x6) accumulates (+=)."""
        V, n = self.cams.V, self.n
        need = L.steepgs_workspace_size(L.STAGE_RENDER_BWD6, n, V) // 4 + 64
        if self.ws_bwd6 is None or self.ws_bwd6.numel() < need:
            self.ws_bwd6 = torch.empty(need, dtype=torch.int32, device=self.dev)
        L.steepgs_render_bwd_split6(params, n, self.sh_degree, self.cams.dev, V, self.cams.opts, self.splats,
                                    self.tiles, self.vals, self.ranges, self.cams.total_tiles,
                                    self.cams.total_pixels, self.image, self.T_final, self.n_contrib, dL_dimage,
                                    target, grads, S, S6, self.ws_bwd6)


def densify6(params: torch.Tensor, sh_degree: int, S6: torch.Tensor, s_scale: float, eps: float,
             eps_split: float = -1e-6, out_capacity: int | None = None):
    """Steepest Density Control over theta = (p, log-scales) on the device:
    S6 [21, n]; the offspring move in position and log-scales."""
    F, n = params.shape
    dev = params.device
    cap = 2 * n if out_capacity is None else int(out_capacity)
    out = torch.empty((F, max(cap, 1)), dtype=torch.float32, device=dev)
    n_out = torch.zeros(1, dtype=torch.int64, device=dev)
    status = torch.zeros(1, dtype=torch.int32, device=dev)
    lam = torch.empty(max(n, 1), dtype=torch.float32, device=dev)
    vmin = torch.empty((6, max(n, 1)), dtype=torch.float32, device=dev)
    split = torch.empty(max(n, 1), dtype=torch.uint8, device=dev)
    ws = torch.empty(L.steepgs_workspace_size(L.STAGE_DENSIFY, n, 1) // 4 + 64, dtype=torch.int32, device=dev)
    L.steepgs_densify6(params, n, sh_degree, S6, s_scale, eps, eps_split, out, cap, n_out, lam, vmin, split, status, ws)
    no = int(n_out.item())
    st = int(status.item())
    return dict(params=out[:, :no] if st == L.OK else None, n_out=no, status=st, lambda_min=lam[:n],
                vmin=vmin[:, :n], split=split[:n])


def densify(params: torch.Tensor, sh_degree: int, S: torch.Tensor, s_scale: float, eps: float,
            eps_split: float = -1e-6, out_capacity: int | None = None, G: torch.Tensor | None = None,
            g_scale: float = 1.0, eps_grad: float = 0.0, budget: int = 0, Gabs: torch.Tensor | None = None,
            adc_tau: float = 0.0):
    """Steepest Density Control on the device; returns the new parameter
    tensor [F, n_out] and the per-Gaussian eigen results.  Reads n_out back.
    Optional: the compactest gate (``G`` [3, n], ``g_scale``, ``eps_grad``),
    the ADC-style gate (``Gabs`` [n], ``g_scale``, ``adc_tau``) and the
    increment budget (``budget``)."""
    F, n = params.shape
    dev = params.device
    cap = 2 * n if out_capacity is None else int(out_capacity)
    out = torch.empty((F, max(cap, 1)), dtype=torch.float32, device=dev)
    n_out = torch.zeros(1, dtype=torch.int64, device=dev)
    status = torch.zeros(1, dtype=torch.int32, device=dev)
    lam = torch.empty(max(n, 1), dtype=torch.float32, device=dev)
    vmin = torch.empty((3, max(n, 1)), dtype=torch.float32, device=dev)
    split = torch.empty(max(n, 1), dtype=torch.uint8, device=dev)
    ws = torch.empty(L.steepgs_workspace_size(L.STAGE_DENSIFY, n, 1) // 4 + 64, dtype=torch.int32, device=dev)
    if G is not None and (G.shape != (3, n) or G.dtype != torch.float32 or not G.is_contiguous()):
        raise ValueError("G must be a contiguous float32 tensor [3, n]")
    if Gabs is not None and (Gabs.shape != (n,) or Gabs.dtype != torch.float32 or not Gabs.is_contiguous()):
        raise ValueError("Gabs must be a contiguous float32 tensor [n]")
    L.steepgs_densify(params, n, sh_degree, S, s_scale, eps, eps_split, out, cap, n_out, lam, vmin, split, status, ws,
                      G=G, g_scale=g_scale, eps_grad=eps_grad, budget=budget, Gabs=Gabs, adc_tau=adc_tau)
    no = int(n_out.item())
    st = int(status.item())
    return dict(params=out[:, :no] if st == L.OK else None, n_out=no, status=st, lambda_min=lam[:n],
                vmin=vmin[:, :n], split=split[:n], out_buffer=out)
