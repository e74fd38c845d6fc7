"""Autotuner for the batched step: tile shape and views per launch.

For a scene (parameters, cameras, targets) it times the HIP-graph-captured
step for every candidate configuration on the device and keeps the fastest.
Candidates: tile shapes 16x16, 16x8 and 8x8 (the library's instantiations)
times views-per-launch groupings (all views in one launch, or groups of a
given size launched back to back with S accumulated, then one densification).

The tile shape changes only how the work is partitioned: a pixel's set of
contributors and their order are fixed by the footprint rule, independent of
tiles, so every candidate computes the same image.
"""
from __future__ import annotations

from dataclasses import dataclass

import torch

from .pipeline import CameraBatch, Rasterizer
from .step import BatchedStep, _Densify
from . import _lib as L

TILE_SHAPES = ((16, 16), (16, 8), (8, 8))


@dataclass
class TuneResult:
    tile: tuple
    views_per_launch: int
    ms: float
    table: list  # (tile, views_per_launch, ms) for every candidate


class GroupedStep:
    """The batched step over groups of views (each group one launch per
    stage), S accumulated over the groups, one densification."""

    def __init__(self, params, sh_degree, scene_cams, opts, target, group, eps, eps_split=-1e-6):
        dev = params.device
        self.params, self.sh_degree, self.eps, self.eps_split = params, sh_degree, eps, eps_split
        F, n = params.shape
        offs = scene_cams.pixel_offsets()
        self.groups = []
        for g0 in range(0, scene_cams.V, group):
            ids = list(range(g0, min(g0 + group, scene_cams.V)))
            cb = CameraBatch(scene_cams.subset(ids), opts, dev)
            lo = 3 * int(offs[ids[0]])
            tg = target[lo: lo + 3 * cb.total_pixels]
            self.groups.append((cb, Rasterizer(cb, sh_degree), tg))
        self.grads = torch.zeros((F, n), dtype=torch.float32, device=dev)
        self.S = torch.zeros((6, n), dtype=torch.float32, device=dev)
        self.dens = _Densify(F, n, dev)
        self.graph = None

    def prepare(self, headroom=1.1):
        for cb, r, _ in self.groups:
            r.project(self.params)
            K = r.sort()
            r._ensure(self.params.shape[1], int(K * headroom) + 4096)

    def run(self):
        self.grads.zero_()
        self.S.zero_()
        for cb, r, tg in self.groups:
            r.project(self.params)
            L.steepgs_sort(r.splats, r.tiles, r.n, cb.V, cb.dev, cb.opts, cb.total_tiles, None, r.vals, r.capacity,
                           r.ranges, r.num, r.status, r.ws_sort, depth_keys=r.dkeys)
            r.render(tg)
            r.backward(self.params, self.grads, self.S, target=tg)
        self.dens.run(self.params, self.sh_degree, self.S, 1.0, self.eps, self.eps_split)

    def capture(self):
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            self.run()
        torch.cuda.synchronize()
        self.graph = g

    def check(self):
        for cb, r, _ in self.groups:
            if int(r.status.item()) != L.OK:
                raise RuntimeError("instance capacity exceeded")
        return self.dens.result()


def _time(fn, reps):
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        fn()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps


def tune(params: torch.Tensor, sh_degree: int, scene_cams, opts: dict, target: torch.Tensor, eps: float = 1e-3,
         tiles=TILE_SHAPES, groups=None, reps: int = 3) -> TuneResult:
    """Time every candidate (graph replays after one warm run) and return the
    fastest.  `groups`: views-per-launch candidates (default: all views, and
    half of them when there are more than two)."""
    V = scene_cams.V
    if groups is None:
        groups = [V] + ([max(1, V // 2)] if V > 2 else [])
    table = []
    for tw, th in tiles:
        o = dict(opts, tile_w=tw, tile_h=th)
        for g in groups:
            if g >= V:
                step = BatchedStep(params, sh_degree, CameraBatch(scene_cams, o, params.device), target, eps=eps)
            else:
                step = GroupedStep(params, sh_degree, scene_cams, o, target, g, eps)
            step.prepare()
            step.run()
            step.check()
            step.capture()
            ms = _time(step.graph.replay, reps)
            step.check()
            table.append(((tw, th), g, ms))
            del step
    best = min(table, key=lambda r: r[2])
    return TuneResult(best[0], best[1], best[2], table)
