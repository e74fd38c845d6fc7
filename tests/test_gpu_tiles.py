"""Tile shapes and the autotuner: the 16x8 and 8x8 kernel instantiations
against the oracle (instance lists bit-exact, image and gradients at the
parity bars), the image bit-identical across tile shapes (a pixel's
contributors do not depend on the tiling), and the autotuner's table."""
import numpy as np
import pytest
import torch

from paper_2505_05587_amd import scenes
from paper_2505_05587_amd.autotune import tune
from tests.gpu_common import check_against, checked_reference, run_gpu, scene_small

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("tile", [(16, 8), (8, 8)])
@pytest.mark.parametrize("kind", ["multiview", "sh3_pinhole", "extreme"])
def test_tile_shape_parity(oracle, kind, tile):
    P, deg, cams, target = scene_small(kind)
    opts = scenes.opts("3dgs", tile_w=tile[0], tile_h=tile[1])
    print(f"\n[case] tile {tile} kind={kind}", flush=True)
    g = run_gpu(P, deg, cams, opts, target=target, want_keys=True)
    keys, vals, ranges = oracle.sort(P, deg, cams, opts)
    assert g["K"] == len(keys)
    np.testing.assert_array_equal(g["keys"], keys)
    np.testing.assert_array_equal(g["vals"], vals)
    np.testing.assert_array_equal(g["ranges"], ranges)
    vref = checked_reference(oracle, P, deg, cams, opts, g, target=target)
    st = check_against(g, vref, cams, f"tile {tile} {kind}")
    assert st["pix_excl"] + st["pix_soft_dev"] < 1e-3
    assert st["gauss_excl"] + st["gauss_soft_dev"] < 1e-2
    # the image does not depend on the tiling
    g16 = run_gpu(P, deg, cams, scenes.opts("3dgs"), target=target)
    np.testing.assert_array_equal(g["image"], g16["image"])
    np.testing.assert_array_equal(g["T_final"], g16["T_final"])
    np.testing.assert_array_equal(g["n_used"], g16["n_used"])


def test_autotuner_table():
    P0, deg, cams, target = scene_small("multiview")
    dev = torch.device("cuda", 0)
    print("\n[case] autotune multiview", flush=True)
    res = tune(torch.from_numpy(P0).to(dev), deg, cams, scenes.opts("3dgs"), torch.from_numpy(target).to(dev),
               groups=[3, 1], reps=2)
    assert len(res.table) == 6
    assert all(ms > 0 for _, _, ms in res.table)
    assert (res.tile, res.views_per_launch, res.ms) in [(t, g, ms) for t, g, ms in res.table]
    assert res.ms == min(ms for _, _, ms in res.table)
