"""One pass of the hot path: project -> sort -> forward (fused L1) -> backward
with splitting matrices -> Steepest Density Control.

``BatchedStep`` runs every view of a camera batch per launch and can be
captured once into a HIP graph (``capture``/``replay``); ``PerViewStep`` issues
the same calls once per view (V = 1), accumulating S over views, and is the
plain form the batched step is compared with.  Both enqueue work only: the
data-dependent sizes live in device memory, capacities are fixed by
``prepare`` and the overflow flags are read back by ``check``.
"""
from __future__ import annotations

import torch

from . import _lib as L
from .pipeline import CameraBatch, Rasterizer


class _Densify:
    def __init__(self, F, n, dev, theta_dim=3):
        self.theta_dim = theta_dim
        self.cap = 2 * n
        self.out = torch.empty((F, max(self.cap, 1)), dtype=torch.float32, device=dev)
        self.n_out = torch.zeros(1, dtype=torch.int64, device=dev)
        self.status = torch.zeros(1, dtype=torch.int32, device=dev)
        self.lam = torch.empty(max(n, 1), dtype=torch.float32, device=dev)
        self.vmin = torch.empty((theta_dim, max(n, 1)), dtype=torch.float32, device=dev)
        self.split = torch.empty(max(n, 1), dtype=torch.uint8, device=dev)
        self.ws = torch.empty(L.steepgs_workspace_size(L.STAGE_DENSIFY, n, 1) // 4 + 64, dtype=torch.int32,
                              device=dev)

    def run(self, params, sh_degree, S, s_scale, eps, eps_split):
        """S: [6, n] (theta = p) or [21, n] (theta = (p, log-scales))"""
        fn = L.steepgs_densify6 if self.theta_dim == 6 else L.steepgs_densify
        fn(params, params.shape[1], sh_degree, S, s_scale, eps, eps_split, self.out, self.cap, self.n_out, self.lam,
           self.vmin, self.split, self.status, self.ws)

    def result(self):
        n_out = int(self.n_out.item())
        if int(self.status.item()) != L.OK:
            raise RuntimeError(f"densify capacity {self.cap} < {n_out}")
        return self.out[:, :n_out]


FORK_CLEARS_RECORDS = 1 << 22


class BatchedStep:
    """theta_dim 3: the splitting matrix over the position (the paper's);
    6: over (position, log-scales), S [21, n] and the dim-6 split."""

    def __init__(self, params: torch.Tensor, sh_degree: int, cams: CameraBatch, target: torch.Tensor,
                 eps: float, eps_split: float = -1e-6, s_scale: float = 1.0, capacity: int = 0, theta_dim: int = 3):
        if theta_dim not in (3, 6):
            raise ValueError("theta_dim is 3 or 6")
        self.params, self.sh_degree, self.cams, self.target = params, sh_degree, cams, target
        self.eps, self.eps_split, self.s_scale = eps, eps_split, s_scale
        self.theta_dim = theta_dim
        F, n = params.shape
        dev = params.device
        self.ras = Rasterizer(cams, sh_degree, capacity)
        self.grads = torch.zeros((F, n), dtype=torch.float32, device=dev)
        self.S = torch.zeros((6 if theta_dim == 3 else 21, n), dtype=torch.float32, device=dev)
        self.dens = _Densify(F, n, dev, theta_dim)
        self.side = torch.cuda.Stream(device=dev)  # default priority
        # side-stream clears from 2^22 records (a 300 MB slot clear) on: below
        # that, the graph's cross-stream dependencies cost more than they hide
        self.fork_clears = cams.V * n >= FORK_CLEARS_RECORDS
        self.graph = None

    def prepare(self, headroom: float = 1.1) -> int:
        """Run the forward once with host checks and fix the instance capacity."""
        self.ras.project(self.params)
        K = self.ras.sort()
        self.ras._ensure(self.params.shape[1], int(K * headroom) + 4096)
        return K

    def run(self):
        r = self.ras
        main = torch.cuda.current_stream()
        r.project(self.params)
        L.steepgs_sort(r.splats, r.tiles, r.n, self.cams.V, self.cams.dev, self.cams.opts, self.cams.total_tiles,
                       None, r.vals, r.capacity, r.ranges, r.num, r.status, r.ws_sort, depth_keys=r.dkeys)
        # the clears of the backward's accumulators read nothing: on large
        # batches they run on a second stream beside the forward blend
        # (VALU-bound, most of the HBM bandwidth free) and join before the
        # backward; on small ones the fork and join cost more than they hide
        if self.fork_clears:
            self.side.wait_stream(main)
            with torch.cuda.stream(self.side):
                self.grads.zero_()
                self.S.zero_()
                if self.theta_dim == 3:
                    r.clear_backward()
        r.render(self.target)
        if self.fork_clears:
            main.wait_stream(self.side)
        else:
            self.grads.zero_()
            self.S.zero_()
        if self.theta_dim == 6:
            r.backward6(self.params, self.grads, self.S, target=self.target)
        else:
            r.backward(self.params, self.grads, self.S, target=self.target, cleared=self.fork_clears)
        self.dens.run(self.params, self.sh_degree, self.S, self.s_scale, self.eps, self.eps_split)

    def capture(self):
        """Capture one step into a HIP graph (after prepare and a warm run)."""
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            self.run()
        torch.cuda.synchronize()
        self.graph = g
        return g

    def replay(self):
        self.graph.replay()

    def check(self):
        """Host-side check of the device status words of the last step."""
        if int(self.ras.status.item()) != L.OK:
            raise RuntimeError(f"instance capacity {self.ras.capacity} < {int(self.ras.num.item())}")
        return self.dens.result()

    @property
    def loss(self):
        return self.ras.loss


class PerViewStep:
    """The same stages issued once per view (V = 1 each), S accumulated over
    the views, then one densification."""

    def __init__(self, params: torch.Tensor, sh_degree: int, scene_cams, opts: dict, target: torch.Tensor,
                 eps: float, eps_split: float = -1e-6, s_scale: float = 1.0, theta_dim: int = 3):
        self.params, self.sh_degree = params, sh_degree
        self.eps, self.eps_split, self.s_scale = eps, eps_split, s_scale
        self.theta_dim = theta_dim
        F, n = params.shape
        dev = params.device
        offs = scene_cams.pixel_offsets()
        self.views = []
        for v in range(scene_cams.V):
            cb = CameraBatch(scene_cams.subset([v]), opts, dev)
            o = 3 * int(offs[v])
            tg = target[o: o + 3 * cb.total_pixels]
            self.views.append((cb, Rasterizer(cb, sh_degree), tg))
        self.grads = torch.zeros((F, n), dtype=torch.float32, device=dev)
        self.S = torch.zeros((6 if theta_dim == 3 else 21, n), dtype=torch.float32, device=dev)
        self.dens = _Densify(F, n, dev, theta_dim)

    def prepare(self, headroom: float = 1.1):
        for cb, r, _ in self.views:
            r.project(self.params)
            K = r.sort()
            r._ensure(self.params.shape[1], int(K * headroom) + 4096)

    def run(self):
        self.grads.zero_()
        self.S.zero_()
        for cb, r, tg in self.views:
            r.project(self.params)
            L.steepgs_sort(r.splats, r.tiles, r.n, 1, cb.dev, cb.opts, cb.total_tiles, None, r.vals, r.capacity,
                           r.ranges, r.num, r.status, r.ws_sort, depth_keys=r.dkeys)
            r.render(tg)
            if self.theta_dim == 6:
                r.backward6(self.params, self.grads, self.S, target=tg)
            else:
                r.backward(self.params, self.grads, self.S, target=tg)
        self.dens.run(self.params, self.sh_degree, self.S, self.s_scale, self.eps, self.eps_split)

    def check(self):
        for cb, r, _ in self.views:
            if int(r.status.item()) != L.OK:
                raise RuntimeError("instance capacity exceeded")
        return self.dens.result()
