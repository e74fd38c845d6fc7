"""The allocation-free forward entry point (scratch in the library's own
device array) against steepgs_render_fwd (scratch in the caller's
workspace), through the C ABI: two calls in a row, the second on a smaller
problem; image, transmittance and counts bit-identical to the workspace form
on the same inputs, the loss equal up to the order of its float sums."""
import numpy as np
import pytest
import torch

from paper_2505_05587_amd import _lib as L
from paper_2505_05587_amd import pipeline, scenes
from tests.gpu_common import scene_small

pytestmark = pytest.mark.gpu


def _forward_both(kind):
    P, deg, cams, target = scene_small(kind)
    opts = scenes.opts("3dgs")
    dev = torch.device("cuda", 0)
    cb = pipeline.CameraBatch(cams, opts, dev)
    ras = pipeline.Rasterizer(cb, deg, capacity=1 << 16)
    Pt = torch.from_numpy(np.ascontiguousarray(P)).to(dev)
    tg = torch.from_numpy(np.ascontiguousarray(target)).to(dev)
    fs = ras.forward(Pt, tg, count_used=True)  # projection, sort and the workspace forward
    torch.cuda.synchronize()
    ref = dict(image=fs.image.clone(), T_final=fs.T_final.clone(), n_contrib=fs.n_contrib.clone(),
               n_used=ras.n_used.clone(), loss=fs.loss.clone())
    Px = cb.total_pixels
    got = dict(image=torch.full((3 * Px,), float("nan"), device=dev),
               T_final=torch.full((Px,), float("nan"), device=dev),
               n_contrib=torch.full((Px,), -1, dtype=torch.int32, device=dev),
               n_used=torch.full((Px,), -1, dtype=torch.int32, device=dev),
               loss=torch.full((cb.V,), float("nan"), device=dev))
    L.steepgs_render_fwd_noalloc(ras.splats, ras.n, ras.vals, ras.ranges, cb.dev, cb.V, cb.opts, cb.total_tiles, Px,
                                 tg, got["image"], got["T_final"], got["n_contrib"], got["n_used"], got["loss"])
    torch.cuda.synchronize()
    return fs.K, ref, got


def test_noalloc_forward_matches_workspace_forward():
    sizes = []
    for kind in ("multiview", "plain_small"):  # the second call is on a smaller problem
        print(f"\n[case] no-alloc forward kind={kind}", flush=True)
        K, ref, got = _forward_both(kind)
        assert K > 0
        for name in ref:
            a = ref[name].cpu().numpy()
            b = got[name].cpu().numpy()
            assert a.shape == b.shape, name
            if name == "loss":
                # per-view sums of per-tile float32 partials added atomically
                # in the order the tiles finish: equal up to that order
                np.testing.assert_allclose(b, a, rtol=1e-6, atol=0)
            else:
                np.testing.assert_array_equal(a.view(np.uint32), b.view(np.uint32), err_msg=name)
        sizes.append(ref["T_final"].numel())
    assert sizes[1] < sizes[0]


def test_noalloc_forward_rejects_bad_arguments():
    o = L.make_opts(scenes.opts("3dgs"))
    lib = L.lib()
    assert lib.steepgs_render_fwd_noalloc(None, -1, None, None, None, 1, o, 1, 1, None, None, None, None, None, None,
                                          None) == L.ERR_INVALID_ARG
