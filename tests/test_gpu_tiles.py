"""Tile shapes and the autotuner: the 16x8 and 8x8 kernel instantiations
against the oracle (instance lists bit-exact, image and gradients at the
parity bars), the image bit-identical across tile shapes (a pixel's
contributors do not depend on the tiling), and the autotuner's table."""
import numpy as np
import pytest
import torch

from paper_2505_05587_amd import scenes
from paper_2505_05587_amd import autotune as AT
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


def test_autotuner_cache_and_parity(oracle, tmp_path):
    # the tuner times its candidates, the cache round-trips the result, and the
    # tuned configuration (tile and launch shape) is parity-green
    P0, deg, cams, target = scene_small("multiview")
    dev = torch.device("cuda", 0)
    print("\n[case] autotune multiview", flush=True)
    opts = scenes.opts("3dgs")
    res = AT.tune(torch.from_numpy(P0).to(dev), deg, cams, opts, torch.from_numpy(target).to(dev), groups=[3, 1],
                  waves=(2, 4), grids=(4, 8), reps=2)
    # stage 1: 3 tiles x 2 groupings; stage 2: the other 3 launch shapes
    assert len(res.table) == 6 + 3
    assert all(ms > 0 for _, ms in res.table)
    assert res.ms == min(ms for _, ms in res.table)
    path = str(tmp_path / "tuned.json")
    key = AT.cache_key(dev, P0.shape[1], cams.V, cams.total_pixels(), deg)
    AT.save(key, res, path)
    back = AT.load(key, path)
    assert (back.tile, back.views_per_launch, back.waves_per_wg, back.wgs_per_cu) == \
        (res.tile, res.views_per_launch, res.waves_per_wg, res.wgs_per_cu)
    assert AT.load("another|key", path) is None
    tuned = back.opts(opts)
    g = run_gpu(P0, deg, cams, tuned, target=target)
    vref = checked_reference(oracle, P0, deg, cams, tuned, g, target=target)
    check_against(g, vref, cams, f"tuned {back.config()}")


@pytest.mark.parametrize("waves,wgs", [(2, 1), (8, 3), (2, 64)])
def test_launch_shapes_give_identical_results(waves, wgs):
    # the launch shape only partitions the work: bit-identical image and
    # counts, gradients and S (fp64 cross-tile sums) for any shape
    P0, deg, cams, target = scene_small("sh3_pinhole")
    print(f"\n[case] launch shape waves={waves} wgs_per_cu={wgs}", flush=True)
    a = run_gpu(P0, deg, cams, scenes.opts("3dgs"), target=target)
    b = run_gpu(P0, deg, cams, scenes.opts("3dgs", raster_waves_per_wg=waves, raster_wgs_per_cu=wgs), target=target)
    for k in ("image", "T_final", "n_used", "grads", "S6"):
        np.testing.assert_array_equal(a[k], b[k], err_msg=k)
