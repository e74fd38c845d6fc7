#!/usr/bin/env python3
"""Benchmark of the SteepGS hot path on one MI355X.

Workload (default): 1,000,000 clustered Gaussians (SH degree 3), 16 views of
mixed resolution -- the batched densification step.  A step is one pass of
project -> sort -> forward with fused L1 -> backward with splitting matrices
-> Steepest Density Control over the whole batch.

The timed region replays the HIP-graph-captured batched step K times
(inputs resident in HBM).  The same step issued per view (V = 1 calls, S
accumulated, then one densification) is timed beside it.  A second pass of K
eager steps records HIP events around every kernel of interest (on the
stream it is launched on) for the per-stage breakdown and the roofline of the
dominant kernel.  The CPU baseline times the FP64 oracle on one view and
scales it to the step.

Prints one JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "ms per fwd+bwd+split step, 1M Gaussians×16 views; batched vs per-view speedup"
PEAK_HBM_GBS = 8000.0
# published fp32 vector peak of MI355X (packed FP32)
PEAK_FP32_TFLOPS = 157.3
# the same without packed-FP32 instructions (this library compiles without
# them): 256 CU x 4 SIMD x 16 lanes x 2 flop (FMA) x 2.4 GHz
PEAK_FP32_NONPACKED_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12
# algorithmic fp32 work of the raster kernels: flops per examined (pixel,
# entry) pair and per contributing pair (quadratic form, exponential and
# tests per examined pair; blend or gradient, moments and sums per
# contributing pair)
FLOP_EXAMINED = 10
FLOP_CONTRIB_FWD = 20
FLOP_CONTRIB_BWD = 60
FLOP_CONTRIB_BWD6 = 83  # + the third and fourth moments of the dim-6 backward


def say(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="batched_16")
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--no-per-view", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--eps", type=float, default=1e-3)
    ap.add_argument("--theta-dim", type=int, choices=(3, 6), default=3,
                    help="splitting matrix over the position (3, the paper's) or position and log-scales (6)")
    ap.add_argument("--no-tune", action="store_true",
                    help="default launch shape instead of the autotuner's (cached per device and shape class)")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="run one plain device copy of this size first (HBM counter calibration under a profiler)")
    return ap.parse_args()


def time_region(fn, steps, torch):
    """Mean ms per step over exactly `steps` calls between two synchronised
    events, the host wall clock of the same region, and the per-step times
    (an event after each step)."""
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    ev[0].record()
    t0 = time.perf_counter()
    for k in range(steps):
        fn()
        ev[k + 1].record()
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) * 1e3 / steps
    per = [ev[k].elapsed_time(ev[k + 1]) for k in range(steps)]
    return ev[0].elapsed_time(ev[steps]) / steps, wall, per


def kernel_times(step, steps, torch, L):
    """K eager steps with HIP events around each timed kernel; returns
    {name: [ms per launch]}"""
    events = {}
    for w in range(len(L.TIMER_NAMES)):
        st = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
        en = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
        for e in st + en:
            e.record()  # creates the underlying event
        events[w] = (st, en)
    torch.cuda.synchronize()
    for w, (st, en) in events.items():
        L.steepgs_set_kernel_timer(w, st, en)
    try:
        for _ in range(steps):
            step.run()
        torch.cuda.synchronize()
    finally:
        for w in events:
            L.steepgs_set_kernel_timer(w, [], [])
    return {L.TIMER_NAMES[w]: [s.elapsed_time(e) for s, e in zip(st, en)] for w, (st, en) in events.items()}


# HBM bytes per launch of each kernel, from rocprofv3 FETCH_SIZE / WRITE_SIZE
# passes over this workload (profiles/hbm_traffic.txt: one line per stage with
# the counter readings in KiB per dispatch, the scale factors from a plain
# 1 GiB device copy and the SHA-256 of the kernel's sources); reported only
# while those sources are unchanged.
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic.txt")
TRAFFIC_WORKLOAD = "batched_16"  # the workload the counter passes profile
KERNEL_SOURCE = {"project": "project.hip", "sort": "sort.hip", "render_fwd": "render_fwd.hip",
                 "render_bwd": "render_bwd.hip", "proj_bwd": "render_bwd.hip", "densify": "densify.hip"}


def _source_digest(stage):
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2505_05587_amd", "csrc")
    for name in (KERNEL_SOURCE[stage], "common.h", "projection.h"):
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(f.read())
    # the record and option layouts every kernel is compiled against
    with open(os.path.join(ROOT, "include", "steepgs.h"), "rb") as f:
        h.update(f.read())
    return h.hexdigest()


def measured_traffic(stage):
    rec = None
    try:
        with open(TRAFFIC_FILE) as f:
            for line in f:
                tok = line.split()
                if len(tok) >= 2 and tok[0] == "stage" and tok[1] == stage:
                    rec = dict(zip(tok[2::2], tok[3::2]))
    except OSError:
        return None
    if not rec or rec.get("sha256") != _source_digest(stage):
        return None
    return int(float(rec["fetch_kib"]) * float(rec["fetch_scale"]) * 1024 +
               float(rec["write_kib"]) * float(rec["write_scale"]) * 1024)


def host_cpu():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def valu_calibration(torch, L, dev):
    """Achievable fp32 VALU rate of plain FMAs (TFLOP/s), best of three
    launches of the library's FMA-loop kernel, timed with events."""
    blocks, iters = torch.cuda.get_device_properties(dev).multi_processor_count * 8, 20000
    out = torch.empty(blocks * 256, dtype=torch.float32, device=dev)
    L.steepgs_calibrate_valu(out, blocks, 100)
    best = None
    for _ in range(3):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        L.steepgs_calibrate_valu(out, blocks, iters)
        b.record()
        torch.cuda.synchronize()
        ms = a.elapsed_time(b)
        best = ms if best is None else min(best, ms)
    return blocks * 256 * iters * 16 / (best * 1e-3) / 1e12


def cpu_baseline(scene, opts):
    """The oracle as it stands on one view of the workload (full Gaussian set),
    scaled to the 16-view step, plus its densification over all Gaussians."""
    import numpy as np
    from oracle import oracle as O
    V = scene.cams.V
    px = scene.cams.pixels()
    v = int(np.argmin(np.abs(px - px.mean())))  # the view closest to the mean resolution
    c1 = scene.cams.subset([v])
    tg = scene.target_view(v).reshape(-1)
    t0 = time.perf_counter()
    r = O.forward_backward(scene.params, scene.sh_degree, c1, opts, tg)
    t_view = time.perf_counter() - t0
    t0 = time.perf_counter()
    O.densify(scene.params, scene.sh_degree, r["S"], 1.0, 1e-3, -1e-6)
    t_dens = time.perf_counter() - t0
    ms = (t_view * px.sum() / px[v] + t_dens) * 1e3
    return {"value": round(ms, 1), "unit": "ms/step", "cores": 1, "kind": "oracle", "host_cpu": host_cpu(),
            "host_nproc": os.cpu_count(),
            "sample": f"view {v} ({int(scene.cams.width[v])}x{int(scene.cams.height[v])}) of {V}, all "
                      f"{scene.n} Gaussians, fwd+bwd+S in {t_view:.1f} s scaled by total/view pixels "
                      f"({px.sum() / px[v]:.2f}x), plus densification of all Gaussians ({t_dens:.1f} s)"}


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: there is no multi-GPU path (views would shard across GPUs with one "
              "all-reduce of gradients and splitting matrices; not implemented). Run with --gpus 1.",
              file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_2505_05587_amd import _lib as L
    from paper_2505_05587_amd import scenes
    from paper_2505_05587_amd.pipeline import CameraBatch
    from paper_2505_05587_amd.step import BatchedStep, PerViewStep

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda", 0)
    say(f"device {torch.cuda.get_device_name(0)}; generating {args.workload}")
    t0 = time.perf_counter()
    scene = scenes.make(args.workload)
    opts = scenes.opts("3dgs")
    say(f"scene ready in {time.perf_counter() - t0:.1f} s: n={scene.n} V={scene.cams.V} px={scene.cams.total_pixels()}")
    if args.copy_mib > 0:
        src = torch.ones(args.copy_mib << 18, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        say(f"calibration copy of {args.copy_mib} MiB done")
        del src, dst
    P = torch.from_numpy(scene.params).to(dev)
    target = torch.from_numpy(scene.target).to(dev)
    # tile and launch shape from the autotuner: its cache entry for this
    # device and shape class, else a tuning pass now (every view in one
    # launch: the batched step is the measured configuration)
    launch = {"source": "default"}
    if not args.no_tune:
        from paper_2505_05587_amd import autotune as AT
        key = AT.cache_key(dev, scene.n, scene.cams.V, scene.cams.total_pixels(), scene.sh_degree)
        tuned = AT.load(key)
        launch = {"source": f"cache {key}"}
        if tuned is None or tuned.views_per_launch != scene.cams.V:
            say(f"tuning the launch shape ({key})")
            tuned = AT.tune(P, scene.sh_degree, scene.cams, opts, target, eps=args.eps, groups=[scene.cams.V])
            launch = {"source": "tuned in this run"}
        opts = tuned.opts(opts)
        launch.update(tuned.config())
        say(f"launch shape: {launch}")
    cams = CameraBatch(scene.cams, opts, dev)

    step = BatchedStep(P, scene.sh_degree, cams, target, eps=args.eps, eps_split=-1e-6, theta_dim=args.theta_dim)
    K = step.prepare()
    say(f"instances K={K} tiles={cams.total_tiles}")
    for _ in range(max(args.warmup, 1)):
        step.run()
    new_params = step.check()
    n_out = new_params.shape[1]
    loss = float(step.loss.sum())
    step.ras.render(target, count_used=True)
    pairs = int(step.ras.n_contrib.to(torch.int64).sum())
    contrib = int(step.ras.n_used.to(torch.int64).sum())
    step.ras.sort(want_counts=True)
    visible = int((step.ras.counts[: cams.V * scene.n] > 0).sum())
    say(f"warm: loss={loss:.5f} n_out={n_out} pairs={pairs} contributors={contrib} visible={visible}")

    use_graph = not args.no_graph
    if use_graph:
        try:
            step.capture()
            step.replay()
            torch.cuda.synchronize()
            step.check()
        except Exception as e:  # graph capture is an optimisation; the eager step is the same work
            say(f"graph capture failed ({e}); timing eager steps")
            use_graph = False
    fn = step.replay if use_graph else step.run
    say(f"timing {args.steps} batched steps ({'graph' if use_graph else 'eager'})")
    torch.cuda.reset_peak_memory_stats()
    ms_batched, wall_batched, per_step = time_region(fn, args.steps, torch)
    peak_gb = torch.cuda.max_memory_allocated() / 2**30
    step.check()
    pct = np.percentile(per_step, [10, 50, 90])
    say(f"batched: {ms_batched:.3f} ms/step (host wall {wall_batched:.3f}; p10/p50/p90 "
        f"{pct[0]:.3f}/{pct[1]:.3f}/{pct[2]:.3f}); peak allocated {peak_gb:.2f} GiB")

    say("per-kernel events over eager steps")
    kt = kernel_times(step, args.steps, torch, L)
    stages = {k: float(np.mean(v)) for k, v in kt.items()}
    say("stages ms: " + ", ".join(f"{k}={v:.3f}" for k, v in stages.items()))

    per_view = None
    if not args.no_per_view:
        step.graph = None
        pv = PerViewStep(P, scene.sh_degree, scene.cams, opts, target, eps=args.eps, eps_split=-1e-6,
                         theta_dim=args.theta_dim)
        pv.prepare()
        for _ in range(max(args.warmup, 1)):
            pv.run()
        pv.check()
        say(f"timing {args.steps} per-view steps")
        per_view, _, _ = time_region(pv.run, args.steps, torch)
        pv.check()
        say(f"per-view: {per_view:.3f} ms/step")
        del pv
        torch.cuda.empty_cache()

    # roofline of the dominant kernel (the raster backward): algorithmic flops
    # per launch / its event-timed duration, against the published fp32 peak,
    # with the non-packed ceiling and the measured FMA-loop rate beside it
    n, V, F = scene.n, scene.cams.V, scene.params.shape[0]
    Px = cams.total_pixels
    valu = valu_calibration(torch, L, dev)
    say(f"FMA-loop VALU rate {valu:.1f} TFLOP/s")
    flops = {
        "render_fwd": pairs * FLOP_EXAMINED + contrib * FLOP_CONTRIB_FWD,
        "render_bwd": pairs * FLOP_EXAMINED + contrib * (FLOP_CONTRIB_BWD if args.theta_dim == 3 else FLOP_CONTRIB_BWD6),
    }
    dom = max(flops, key=lambda k: stages[k])
    achieved = flops[dom] / (stages[dom] * 1e-3) / 1e12
    roof = {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
            "frac": round(achieved / PEAK_FP32_TFLOPS, 4),
            # the counter passes profile the default (dim-3) kernels only
            "traffic": (measured_traffic(dom) if args.theta_dim == 3 and args.workload == TRAFFIC_WORKLOAD
                        else None),
            "kernel": dom, "ms": round(stages[dom], 4), "flop_per_launch": flops[dom],
            "peak_nonpacked": round(PEAK_FP32_NONPACKED_TFLOPS, 1),
            "frac_nonpacked": round(achieved / PEAK_FP32_NONPACKED_TFLOPS, 4),
            "valu_fma_loop_measured": round(valu, 1), "frac_of_measured": round(achieved / valu, 4)}
    other = [k for k in flops if k != dom][0]
    roof["other_raster"] = {"kernel": other, "achieved": round(flops[other] / (stages[other] * 1e-3) / 1e12, 3),
                            "frac": round(flops[other] / (stages[other] * 1e-3) / 1e12 / PEAK_FP32_TFLOPS, 4)}
    # HBM fraction of the memory-bound stages: compulsory bytes (each array
    # read or written once per stage) / event-timed stage duration / 8 TB/s
    Tt = cams.total_tiles
    Nv = visible
    B = {
        "project": n * 4 * F + Nv * 52,
        "sort": Nv * 16 + K * 24 + K * 8 + K * 12 + Tt * 8,
        "proj_bwd": n * 4 * F + Nv * (36 + 52) + n * 4 * F + n * 24 + n * 24,
        "densify": n * (4 * F + 24) + n * 17 + n_out * 4 * F,
    }
    hbm = {k: {"bytes": int(b), "GB/s": round(b / (stages[k] * 1e-3) / 1e9, 1),
               "frac": round(b / (stages[k] * 1e-3) / 1e9 / PEAK_HBM_GBS, 4)} for k, b in B.items()}

    cpu = None
    if not args.no_cpu_baseline:
        say("CPU baseline: oracle on one view")
        cpu = cpu_baseline(scene, opts)
        say(f"cpu baseline {cpu['value']} ms/step")

    out = {
        "metric": METRIC,
        "value": round(ms_batched, 4),
        "unit": "ms/step",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_batched, 4),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": args.workload, "gaussians": n, "views": V, "pixels": Px, "sh_degree": scene.sh_degree,
                   "resolutions": [f"{w}x{h}" for w, h in zip(cams.widths, cams.heights)],
                   "tile": f"{opts['tile_w']}x{opts['tile_h']}", "graph": use_graph, "eps_split": -1e-6,
                   "theta_dim": args.theta_dim, "launch": launch},
        "step_ms_p10_p50_p90": [round(float(x), 4) for x in pct],
        "peak_allocated_gib": round(peak_gb, 3),
        "per_view_ms_per_step": None if per_view is None else round(per_view, 4),
        "speedup_batched_vs_per_view": None if per_view is None else round(per_view / ms_batched, 3),
        "stages_ms": {k: round(v, 4) for k, v in stages.items()},
        "counts": {"instances": K, "visible_pairs": visible, "examined_pairs": pairs, "contributing_pairs": contrib,
                   "n_out": n_out, "loss": round(loss, 6)},
        "roofline": roof,
        "hbm_frac": hbm,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
