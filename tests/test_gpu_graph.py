"""The batched step captured in a HIP graph gives the eager step's results on
every replay, with unrelated eager work and synchronisations between the
replays: instance list and image bit-identical, loss, gradients and S within
the reordering of float atomics, the same split decisions where lambda_min is
clear of the threshold.  The backward run on slots cleared ahead of it (on
another stream) equals the backward that clears them itself."""
import numpy as np
import pytest
import torch

from paper_2505_05587_amd import scenes
from paper_2505_05587_amd.pipeline import CameraBatch
from paper_2505_05587_amd.step import BatchedStep
from tests.gpu_common import assert_group_close, s6_to_mats, scene_small

pytestmark = pytest.mark.gpu


def _snapshot(step):
    r = step.ras
    K = int(r.num.item())
    new = step.check()
    return dict(K=K, vals=r.vals[:K].cpu().numpy().copy(), ranges=r.ranges.cpu().numpy().copy(),
                image=r.image.cpu().numpy().copy(), loss=r.loss.cpu().numpy().copy(),
                grads=step.grads.cpu().numpy().astype(np.float64), S=step.S.cpu().numpy().astype(np.float64),
                lam=step.dens.lam.cpu().numpy().astype(np.float64), split=step.dens.split.cpu().numpy().copy(),
                new=new.cpu().numpy().copy())


@pytest.mark.parametrize("fork", [False, True])
@pytest.mark.parametrize("kind", ["multiview", "sh3_pinhole"])
def test_graph_replays_match_eager(kind, fork):
    # fork: the accumulators cleared on a second stream beside the forward
    # blend (the large-batch path), forced on this small scene
    P0, deg, cams, target = scene_small(kind)
    print(f"\n[case] graph replay kind={kind} fork={fork}", flush=True)
    dev = torch.device("cuda", 0)
    opts = scenes.opts("3dgs")
    step = BatchedStep(torch.from_numpy(P0).to(dev), deg, CameraBatch(cams, opts, dev),
                       torch.from_numpy(target).to(dev), eps=1e-3, eps_split=-1e-6)
    step.fork_clears = fork
    step.prepare()
    step.run()
    torch.cuda.synchronize()
    ref = _snapshot(step)
    step.capture()
    rng = torch.Generator(device=dev).manual_seed(5)
    n = P0.shape[1]
    for rep in range(3):
        # unrelated eager work between replays
        a = torch.randn(512, 512, device=dev, generator=rng)
        (a @ a).sum().item()
        step.S.fill_(123.0)
        step.grads.fill_(-7.0)
        step.ras.ws_bwd.fill_(0x3FF00000)  # the backward's moment slots: nonzero doubles
        step.replay()
        torch.cuda.synchronize()
        got = _snapshot(step)
        assert got["K"] == ref["K"]
        np.testing.assert_array_equal(got["vals"], ref["vals"])
        np.testing.assert_array_equal(got["ranges"], ref["ranges"])
        np.testing.assert_array_equal(got["image"], ref["image"])
        np.testing.assert_allclose(got["loss"], ref["loss"], rtol=1e-5)  # summed with float atomics
        assert_group_close(got["grads"], ref["grads"], np.zeros(n, bool), rel=1e-4, abs_frac=1e-6,
                           what=f"replay {rep}")
        Mg, Mr = s6_to_mats(got["S"]), s6_to_mats(ref["S"])
        d = np.linalg.norm((Mg - Mr).reshape(n, -1), axis=1)
        r = np.linalg.norm(Mr.reshape(n, -1), axis=1)
        assert (d <= 1e-4 * r + 1e-6 * r.max()).all(), f"replay {rep}: S differs"
        sure = np.abs(ref["lam"] + 1e-6) > 1e-4 * r + 1e-12
        np.testing.assert_array_equal(got["split"][sure], ref["split"][sure])
        if np.array_equal(got["split"], ref["split"]):
            assert got["new"].shape == ref["new"].shape


def test_per_view_form_matches_batched():
    # the same five calls issued once per view (V = 1 each, S accumulated)
    # against the batched step over all views: images and transmittance
    # bit-identical per view, losses per view, gradients and S within the
    # reordering of float sums, the same split decisions where lambda_min is
    # clear of the threshold
    from paper_2505_05587_amd.step import PerViewStep
    P0, deg, cams, target = scene_small("multiview")
    print("\n[case] per-view form vs batched, multiview", flush=True)
    dev = torch.device("cuda", 0)
    opts = scenes.opts("3dgs")
    P = torch.from_numpy(P0).to(dev)
    tg = torch.from_numpy(target).to(dev)
    bat = BatchedStep(P, deg, CameraBatch(cams, opts, dev), tg, eps=1e-3, eps_split=-1e-6)
    bat.prepare()
    bat.run()
    pv = PerViewStep(P, deg, cams, opts, tg, eps=1e-3, eps_split=-1e-6)
    pv.prepare()
    pv.run()
    torch.cuda.synchronize()
    n = P0.shape[1]
    offs = cams.pixel_offsets()
    img_b = bat.ras.image.cpu().numpy()
    T_b = bat.ras.T_final.cpu().numpy()
    loss_b = bat.ras.loss.cpu().numpy()
    for v, (cb, r, _) in enumerate(pv.views):
        npx = cb.total_pixels
        np.testing.assert_array_equal(r.image.cpu().numpy(), img_b[3 * offs[v]: 3 * offs[v] + 3 * npx])
        np.testing.assert_array_equal(r.T_final.cpu().numpy(), T_b[offs[v]: offs[v] + npx])
        np.testing.assert_allclose(r.loss.cpu().numpy()[0], loss_b[v], rtol=1e-5)  # summed with float atomics
    gb = bat.grads.cpu().numpy().astype(np.float64)
    gp = pv.grads.cpu().numpy().astype(np.float64)
    assert_group_close(gp, gb, np.zeros(n, bool), rel=1e-4, abs_frac=1e-6, what="per-view vs batched")
    Mb, Mp = s6_to_mats(bat.S.cpu().numpy().astype(np.float64)), s6_to_mats(pv.S.cpu().numpy().astype(np.float64))
    d = np.linalg.norm((Mp - Mb).reshape(n, -1), axis=1)
    r = np.linalg.norm(Mb.reshape(n, -1), axis=1)
    assert (d <= 1e-4 * r + 1e-6 * r.max()).all()
    lam_b = bat.dens.lam[:n].cpu().numpy().astype(np.float64)
    sure = np.abs(lam_b + 1e-6) > 1e-4 * r + 1e-12
    np.testing.assert_array_equal(pv.dens.split[:n].cpu().numpy()[sure], bat.dens.split[:n].cpu().numpy()[sure])


@pytest.mark.parametrize("side", [False, True])
def test_backward_on_cleared_slots_matches_split(side):
    # steepgs_render_bwd_clear (same stream, or a second stream joined by an
    # event) then steepgs_render_bwd_split_cleared: gradients, S and the
    # per-pair 2D gradients bit-identical to steepgs_render_bwd_split, with
    # the slots poisoned before the clear
    from paper_2505_05587_amd.pipeline import Rasterizer
    P0, deg, cams, target = scene_small("multiview")
    print(f"\n[case] backward on cleared slots, side stream={side}", flush=True)
    dev = torch.device("cuda", 0)
    opts = scenes.opts("3dgs")
    cb = CameraBatch(cams, opts, dev)
    P = torch.from_numpy(P0).to(dev)
    tg = torch.from_numpy(target).to(dev)
    r = Rasterizer(cb, deg)
    r.forward(P, target=tg)
    F, n = P.shape
    out = []
    for cleared in (False, True):
        grads = torch.zeros((F, n), dtype=torch.float32, device=dev)
        S = torch.zeros((6, n), dtype=torch.float32, device=dev)
        r.ws_bwd.fill_(0x3FF00000)
        if cleared:
            if side:
                other = torch.cuda.Stream(device=dev)
                other.wait_stream(torch.cuda.current_stream())
                with torch.cuda.stream(other):
                    r.clear_backward()
                torch.cuda.current_stream().wait_stream(other)
            else:
                r.clear_backward()
        r.backward(P, grads, S, target=tg, keep_grad2d=True, cleared=cleared)
        torch.cuda.synchronize()
        out.append((grads.cpu().numpy(), S.cpu().numpy(), r.grad2d.cpu().numpy().copy()))
    for a, b in zip(out[0], out[1]):
        np.testing.assert_array_equal(a, b)
    assert np.abs(out[0][1]).max() > 0

