"""GPU runs of the two 3M-Gaussian workloads, checked at sampled outputs and
by properties that hold at any size.

* ``autograd_4k`` (3,000,000 Gaussians, 4 views at 1920x1080): the autograd
  wrapper's forward + torch L1 loss + backward, with time per step and peak
  memory printed; sampled pixels and sampled Gaussians' gradients and S_i
  against the oracle.
* ``densify_32`` (3,000,000 Gaussians, 32 views of mixed resolution): the
  batched step with S_i summed over all views, then the split; the split set
  checked against the oracle's densification of the same S (sure decisions),
  the offspring layout and sampled pixels of two views against the oracle.
"""
import numpy as np
import pytest
import torch

from paper_2505_05587_amd import scenes
from paper_2505_05587_amd.autograd import SplatRenderer, l1_loss
from paper_2505_05587_amd.pipeline import CameraBatch
from paper_2505_05587_amd.step import BatchedStep
from tests.gpu_common import sample_gaussians, sampled_check

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[large] {msg}", flush=True)


def _pixels(oracle, cams, P, deg, opts, image, rng, count):
    Px = cams.total_pixels()
    pix = np.sort(rng.choice(Px, size=count, replace=False))
    rgb, _, amb = oracle.render_pixels(P, deg, cams, opts, pix)
    offs = cams.pixel_offsets()
    got = np.zeros((count, 3))
    for k, p in enumerate(pix):
        v = int(np.searchsorted(offs, p, side="right") - 1)
        plane = int(cams.width[v]) * int(cams.height[v])
        for ch in range(3):
            got[k, ch] = image[3 * offs[v] + ch * plane + (p - offs[v])]
    ok = (np.abs(got - rgb) <= 1e-5 + 1e-4 * np.abs(rgb)).all(axis=1) | amb
    assert ok.all(), f"{(~ok).sum()} of {count} sampled pixels out of tolerance"


def test_autograd_4k(oracle):
    s = scenes.autograd_4k()
    opts = scenes.opts("3dgs")
    dev = torch.device("cuda", 0)
    print(f"\n[case] autograd_4k n={s.n} V={s.cams.V}", flush=True)
    rend = SplatRenderer(CameraBatch(s.cams, opts, dev), s.sh_degree)
    P = torch.from_numpy(s.params).to(dev).requires_grad_(True)
    tg = torch.from_numpy(s.target).to(dev)
    S = torch.zeros((6, s.n), dtype=torch.float32, device=dev)
    for _ in range(2):  # warm-up (buffers, instance capacity)
        P.grad = None
        S.zero_()
        l1_loss(rend, rend.render(P, S), tg).backward()
    torch.cuda.synchronize()
    torch.cuda.reset_peak_memory_stats()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    P.grad = None
    S.zero_()
    a.record()
    img = rend.render(P, S)
    loss = l1_loss(rend, img, tg)
    loss.backward()
    b.record()
    torch.cuda.synchronize()
    _say(f"fwd+bwd+S {a.elapsed_time(b):.2f} ms, peak allocated {torch.cuda.max_memory_allocated() / 2**30:.2f} GiB, "
         f"instances {int(rend.ras.num.item())}")
    rng = np.random.default_rng(21)
    _say("sampled pixels")
    _pixels(oracle, s.cams, s.params, s.sh_degree, opts, img.detach().cpu().numpy().astype(np.float64), rng, 600)
    _say("sampled gradients")
    rend.ras.render(tg, count_used=True)
    torch.cuda.synchronize()
    gids, info = sample_gaussians(oracle, s, opts, rng, heavy_tiles=0, needles=4, random=12)
    st = sampled_check(oracle, s, opts, img.detach().cpu().numpy().astype(np.float64), rend.ras.n_used.cpu().numpy(),
                       P.grad.detach().cpu().numpy().astype(np.float64), S.cpu().numpy().astype(np.float64), gids,
                       "autograd_4k")
    assert st["excluded"] + st["soft_dev"] <= 0.2


def test_densify_32(oracle):
    s = scenes.densify_32()
    opts = scenes.opts("3dgs")
    dev = torch.device("cuda", 0)
    print(f"\n[case] densify_32 n={s.n} V={s.cams.V}", flush=True)
    step = BatchedStep(torch.from_numpy(s.params).to(dev), s.sh_degree, CameraBatch(s.cams, opts, dev),
                       torch.from_numpy(s.target).to(dev), eps=1e-3, eps_split=-1e-6)
    K = step.prepare()
    step.run()
    new = step.check()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    step.run()
    b.record()
    new = step.check()
    torch.cuda.synchronize()
    split = step.dens.split[: s.n].cpu().numpy().astype(bool)
    _say(f"step {a.elapsed_time(b):.2f} ms, instances {K}, splits {split.sum()}, n_out {new.shape[1]}")
    # the split against the oracle's densification of the same S
    S6 = step.S.cpu().numpy().astype(np.float64)
    S9 = np.stack([S6[[0, 1, 2]], S6[[1, 3, 4]], S6[[2, 4, 5]]]).reshape(9, s.n)
    _say("oracle densify")
    ref = oracle.densify(s.params, s.sh_degree, S9, 1.0, 1e-3, -1e-6)
    Sn = np.linalg.norm(S9, axis=0)
    sure = np.abs(ref["lambda_min"] + 1e-6) > 1e-4 * Sn
    np.testing.assert_array_equal(split[sure], ref["split"][sure])
    assert abs(int(split.sum()) - int(ref["split"].sum())) <= int((~sure).sum())
    assert new.shape[1] == s.n + split.sum()
    # S summed over all 32 views and the gradients of sampled Gaussians against
    # the oracle's (Algorithm 1's densification reads this accumulated S),
    # the in-band decisions of their pixels resolved; and their split
    # decisions on the oracle's own S
    _say("sampled S and gradients over 32 views")
    step.ras.render(step.target, count_used=True)
    torch.cuda.synchronize()
    rng_s = np.random.default_rng(23)
    gids, info = sample_gaussians(oracle, s, opts, rng_s, heavy_tiles=0, needles=4, random=12)
    st = sampled_check(oracle, s, opts, step.ras.image.cpu().numpy().astype(np.float64),
                       step.ras.n_used.cpu().numpy(), step.grads.cpu().numpy().astype(np.float64), S6, gids,
                       "densify_32")
    assert st["excluded"] + st["soft_dev"] <= 0.2
    _, S_ref, _ = oracle.grads_sampled(s.params, s.sh_degree, s.cams, opts, s.target, gids)
    ref_s = oracle.densify(s.params[:, gids], s.sh_degree, S_ref.T.copy(), 1.0, 1e-3, -1e-6)
    Sn_s = np.linalg.norm(S_ref, axis=1)
    sure_s = np.abs(ref_s["lambda_min"] + 1e-6) > 1e-4 * Sn_s
    np.testing.assert_array_equal(split[gids][sure_s], ref_s["split"][sure_s])
    # sampled pixels of two views against the oracle on those views alone
    rng = np.random.default_rng(22)
    views = [0, 17]
    sub = s.cams.subset(views)
    offs = s.cams.pixel_offsets()
    img = step.ras.image.cpu().numpy().astype(np.float64)
    parts = [img[3 * offs[v]: 3 * offs[v] + 3 * int(s.cams.width[v] * s.cams.height[v])] for v in views]
    _say("sampled pixels")
    _pixels(oracle, sub, s.params, s.sh_degree, opts, np.concatenate(parts), rng, 500)
