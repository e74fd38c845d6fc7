"""Autotuner of the batched step's launch shape, with a JSON cache.

For a scene (parameters, cameras, targets) it times the HIP-graph-captured
step for candidate configurations on the device and keeps the fastest:

- tile shape: 16x16, 16x8 and 8x8 (the library's instantiations);
- views per launch: all views in one launch, or groups launched back to back
  with S accumulated, then one densification;
- persistent raster grid: workgroups per compute unit of the forward and
  backward blend kernels (their atomic tile queue hands out the work, so
  the grid only sets how many wavefronts compete for it);
- wavefronts per workgroup of those kernels (each wavefront works on a tile
  of its own; the workgroup size sets the dispatch granularity and the LDS
  block per workgroup).

The search is staged: tile shape x views per launch at the default launch
shape, then the launch shape for the best of those.  The LDS staging batch
of the raster kernels is fixed at 64 entries, one per lane of the wavefront
that stages them.  None of these choices changes any result: a pixel's
contributors and their order are fixed by the footprint rule, independent of
tiles and launch shape (the GPU tests check the tuned configuration against
the oracle).

Results are cached in a JSON file keyed by device and shape class (Gaussian
count, views, pixels and SH degree on a log2 scale); ``python -m
paper_2505_05587_amd.autotune --workload batched_16 --out FILE`` tunes a
workload and writes its entry.
"""
from __future__ import annotations

import json
import math
import os
from dataclasses import asdict, dataclass, field

import torch

from . import _lib as L
from .pipeline import CameraBatch, Rasterizer
from .step import BatchedStep, _Densify

TILE_SHAPES = ((16, 16), (16, 8), (8, 8))
WAVES_PER_WG = (2, 4, 8)
WGS_PER_CU = (4, 6, 8, 12)
CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned_configs.json")


@dataclass
class TuneResult:
    tile: tuple
    views_per_launch: int
    waves_per_wg: int
    wgs_per_cu: int
    ms: float
    table: list = field(default_factory=list)  # [config dict, ms] of every candidate

    def opts(self, base: dict) -> dict:
        """`base` raster options with the tuned tile and launch shape"""
        return dict(base, tile_w=self.tile[0], tile_h=self.tile[1], raster_waves_per_wg=self.waves_per_wg,
                    raster_wgs_per_cu=self.wgs_per_cu)

    def config(self) -> dict:
        return {"tile": f"{self.tile[0]}x{self.tile[1]}", "views_per_launch": self.views_per_launch,
                "waves_per_wg": self.waves_per_wg, "wgs_per_cu": self.wgs_per_cu, "ms": round(self.ms, 4)}


def shape_class(n: int, V: int, pixels: int, sh_degree: int) -> str:
    lg = lambda x: int(round(math.log2(max(int(x), 1))))  # noqa: E731
    return f"n2^{lg(n)}_V{V}_px2^{lg(pixels)}_sh{sh_degree}"


def cache_key(device, n: int, V: int, pixels: int, sh_degree: int) -> str:
    props = torch.cuda.get_device_properties(device)
    arch = getattr(props, "gcnArchName", "") or props.name
    return f"{arch.split(':')[0]}|{props.multi_processor_count}cu|{shape_class(n, V, pixels, sh_degree)}"


def load(key: str, path: str = CACHE) -> TuneResult | None:
    try:
        with open(path) as f:
            d = json.load(f).get(key)
    except (OSError, ValueError):
        return None
    if not d:
        return None
    return TuneResult(tuple(d["tile"]), int(d["views_per_launch"]), int(d["waves_per_wg"]), int(d["wgs_per_cu"]),
                      float(d["ms"]), d.get("table", []))


def save(key: str, res: TuneResult, path: str = CACHE) -> None:
    try:
        with open(path) as f:
            allk = json.load(f)
    except (OSError, ValueError):
        allk = {}
    allk[key] = asdict(res)
    with open(path, "w") as f:
        json.dump(allk, f, indent=1, sort_keys=True)


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

    def camera_batches(self):
        return [cb for cb, _, _ in self.groups]

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


def _set_launch(cbs, waves, wgs):
    for cb in cbs:
        cb.opts.raster_waves_per_wg = waves
        cb.opts.raster_wgs_per_cu = wgs


def tune(params: torch.Tensor, sh_degree: int, scene_cams, opts: dict, target: torch.Tensor, eps: float = 1e-3,
         tiles=TILE_SHAPES, groups=None, waves=WAVES_PER_WG, grids=WGS_PER_CU, reps: int = 3) -> TuneResult:
    """Time the candidates (graph replays after one warm run) and return the
    fastest.  `groups`: views-per-launch candidates (default: all views, and
    half of them when there are more than two)."""
    V = scene_cams.V
    if groups is None:
        groups = [V] + ([max(1, V // 2)] if V > 2 else [])
    table = []

    def build(tile, g):
        o = dict(opts, tile_w=tile[0], tile_h=tile[1])
        if g >= V:
            step = BatchedStep(params, sh_degree, CameraBatch(scene_cams, o, params.device), target, eps=eps)
            cbs = [step.cams]
        else:
            step = GroupedStep(params, sh_degree, scene_cams, o, target, g, eps)
            cbs = step.camera_batches()
        step.prepare()
        return step, cbs

    def measure(step, cbs, tile, g, w, k):
        _set_launch(cbs, w, k)
        step.run()
        step.check()
        step.capture()
        ms = _time(step.graph.replay, reps)
        step.check()
        table.append([{"tile": list(tile), "views_per_launch": g, "waves_per_wg": w, "wgs_per_cu": k}, ms])
        return ms

    # stage 1: tile shape x views per launch at the default launch shape
    best1 = None
    for tile in tiles:
        for g in groups:
            step, cbs = build(tile, g)
            ms = measure(step, cbs, tile, g, 4, 8)
            if best1 is None or ms < best1[2]:
                best1 = (tile, g, ms)
            del step
    # stage 2: launch shape of the raster kernels for the best of those
    tile, g, _ = best1
    step, cbs = build(tile, g)
    best = (4, 8, best1[2])
    for w in waves:
        for k in grids:
            if (w, k) == (4, 8):
                continue
            ms = measure(step, cbs, tile, g, w, k)
            if ms < best[2]:
                best = (w, k, ms)
    del step
    return TuneResult(tuple(tile), g, best[0], best[1], best[2], table)


def main():
    import argparse

    from . import scenes
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--workload", default="batched_16")
    ap.add_argument("--out", default=CACHE)
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--all-views", action="store_true", help="tune with every view in one launch only")
    args = ap.parse_args()
    dev = torch.device("cuda", 0)
    scene = scenes.make(args.workload)
    P = torch.from_numpy(scene.params).to(dev)
    tg = torch.from_numpy(scene.target).to(dev)
    res = tune(P, scene.sh_degree, scene.cams, scenes.opts("3dgs"), tg, reps=args.reps,
               groups=[scene.cams.V] if args.all_views else None)
    key = cache_key(dev, scene.n, scene.cams.V, scene.cams.total_pixels(), scene.sh_degree)
    save(key, res, args.out)
    print(json.dumps({"key": key, **res.config()}))


if __name__ == "__main__":
    main()
