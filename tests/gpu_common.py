"""Helpers of the GPU parity tests: run the HIP path through the C ABI and
compare with the oracle at the stated tolerances."""
import numpy as np
import torch

from paper_2505_05587_amd import pipeline
from paper_2505_05587_amd import scenes

# per-parameter-group rows of the planar layout
GROUPS = {"mean": slice(0, 3), "log_scale": slice(3, 6), "quat": slice(6, 10), "opacity": slice(10, 11),
          "sh": slice(11, None)}


def run_gpu(params, sh_degree, cams, opts, target=None, backward=True, want_keys=False, keep_grad2d=False):
    dev = torch.device("cuda", 0)
    cb = pipeline.CameraBatch(cams, opts, dev)
    ras = pipeline.Rasterizer(cb, sh_degree, capacity=1024)
    P = torch.from_numpy(np.ascontiguousarray(params)).to(dev)
    tg = None if target is None else torch.from_numpy(np.ascontiguousarray(target)).to(dev)
    fs = ras.forward(P, tg, want_keys=want_keys, count_used=True, want_counts=True)
    out = dict(K=fs.K, image=fs.image.cpu().numpy().astype(np.float64), T_final=fs.T_final.cpu().numpy(),
               n_contrib=fs.n_contrib.cpu().numpy(), n_used=ras.n_used.cpu().numpy(), splats=ras.splats.cpu().numpy(),
               tiles=ras.counts[: cams.V * P.shape[1]].cpu().numpy().view(np.uint32),
               rect_tiles=ras.tiles.cpu().numpy().view(np.uint32), vals=ras.vals[: fs.K].cpu().numpy().view(np.uint32),
               ranges=ras.ranges.cpu().numpy().view(np.uint32).reshape(-1, 2))
    if want_keys:
        out["keys"] = ras.keys[: fs.K].cpu().numpy().view(np.uint64)
    if tg is not None:
        out["loss"] = fs.loss.cpu().numpy().astype(np.float64)
        if backward:
            grads = torch.zeros_like(P)
            S = torch.zeros((6, P.shape[1]), dtype=torch.float32, device=dev)
            ras.backward(P, grads, S, target=tg, keep_grad2d=keep_grad2d)
            out["grads"] = grads.cpu().numpy().astype(np.float64)
            out["S6"] = S.cpu().numpy().astype(np.float64)
            if keep_grad2d:
                slots = ras.grad2d[: 12 * cams.V * P.shape[1]].view(-1, 12)
                out["grad2d"] = slots[:, :9].t().contiguous().cpu().numpy()  # [9][V*n]
    torch.cuda.synchronize()
    return out


def s9_to_s6(S9):
    """oracle [9][n] row-major 3x3 -> [6][n] xx xy xz yy yz zz"""
    return S9[[0, 1, 2, 4, 5, 8]]


def s6_to_mats(S6):
    n = S6.shape[1]
    M = np.zeros((n, 3, 3))
    idx = [(0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2)]
    for k, (a, b) in enumerate(idx):
        M[:, a, b] = S6[k]
        M[:, b, a] = S6[k]
    return M


def _report(what, dn, tol, rn, gross):
    i = int(np.argmax(dn / np.maximum(tol, 1e-300)))
    extra = ""
    if gross is not None:
        extra = f" gross/|ref|={gross[i] / max(rn[i], 1e-300):.1f}"
    return f"worst |d|={dn[i]:.3e} |ref|={rn[i]:.3e} tol={tol[i]:.3e}{extra}"


def assert_group_close(got, ref, exclude, rel=1e-3, abs_frac=1e-6, what="", gross=None):
    """Per Gaussian and parameter group: |d| <= rel*|ref| + abs_frac*max_i |ref_i|
    (Euclidean norms over the group's rows).  ``gross`` (the oracle's gross
    magnitudes of the summed terms) only annotates a failure.  Returns the
    largest |d| / tol."""
    keep = ~exclude
    worst = 0.0
    for name, sl in GROUPS.items():
        g = got[sl][:, keep]
        r = ref[sl][:, keep]
        if r.size == 0:
            continue
        dn = np.linalg.norm(g - r, axis=0)
        rn = np.linalg.norm(r, axis=0)
        tol = rel * rn + abs_frac * rn.max()
        gn = None if gross is None else np.linalg.norm(gross[sl][:, keep], axis=0)
        bad = dn > tol
        if bad.any():
            raise AssertionError(f"{what} group {name}: {bad.sum()} of {bad.size} Gaussians out of tolerance; "
                                 + _report(what, dn, tol, rn, gn))
        worst = max(worst, float(np.max(dn / np.maximum(tol, 1e-300))))
    print(f"[bar] {what} gradients: worst |d|/tol = {worst:.3f}", flush=True)
    return worst


def assert_S_close(S6_gpu, S9_ref, exclude, rel=1e-3, abs_frac=1e-6, gross=None, what=""):
    """Per Gaussian: Frobenius |S_gpu - S_ref| <= rel*|S_ref| + abs_frac*max_i |S_ref_i|."""
    ref = s9_to_s6(S9_ref)
    keep = ~exclude
    M_g = s6_to_mats(S6_gpu)[keep]
    M_r = s6_to_mats(ref)[keep]
    dn = np.linalg.norm((M_g - M_r).reshape(len(M_g), -1), axis=1)
    rn = np.linalg.norm(M_r.reshape(len(M_r), -1), axis=1)
    if rn.size == 0:
        return 0.0
    tol = rel * rn + abs_frac * rn.max()
    gn = None if gross is None else np.linalg.norm(gross[:, keep], axis=0)
    bad = dn > tol
    assert not bad.any(), f"{what} S: {bad.sum()} of {bad.size} out of tolerance; " + _report(what, dn, tol, rn, gn)
    worst = float(np.max(dn / np.maximum(tol, 1e-300)))
    print(f"[bar] {what} S: worst |d|/tol = {worst:.3f}", flush=True)
    return worst


def image_close(img_gpu, img_ref, pix_exclude_rgb=None, atol=1e-5, rtol=1e-4):
    d = np.abs(img_gpu - img_ref)
    ok = d <= atol + rtol * np.abs(img_ref)
    if pix_exclude_rgb is not None:
        ok |= pix_exclude_rgb
    return ok


def expand_pixel_mask(mask_px, cams):
    """[Px] pixel mask -> packed [3*Px] image mask (per view planar)."""
    out = []
    offs = cams.pixel_offsets()
    for v in range(cams.V):
        npx = int(cams.width[v] * cams.height[v])
        m = mask_px[offs[v]: offs[v] + npx]
        out.append(np.tile(m, 3))
    return np.concatenate(out)


def scene_small(kind, seed=0):
    """small parity scenes of several shapes"""
    if kind == "plain_small":
        s = scenes.plain_small()
        return s.params, s.sh_degree, s.cams, s.target
    rng = np.random.default_rng(100 + seed)
    if kind == "sh3_pinhole":
        P = scenes.clustered_gaussians(rng, 3000, 40, sh_degree=3, log_scale_mu=-3.5, log_scale_sigma=0.6,
                                       cluster_std=0.2, extent=1.0)
        cams = scenes.make_cameras([(0.3, -0.4, 3.2)], [(150, 110)])
        return P, 3, cams, scenes.smooth_target(rng, cams, 10)
    if kind == "multiview":
        P = scenes.clustered_gaussians(rng, 4000, 50, sh_degree=2, log_scale_mu=-3.8, log_scale_sigma=0.8,
                                       cluster_std=0.2, extent=1.0, powerlaw=1.5)
        pos = scenes.sphere_positions(rng, 3, 3.5, upper_only=True)
        cams = scenes.make_cameras(pos, [(97, 61), (64, 64), (130, 45)])
        return P, 2, cams, scenes.uniform_target(rng, cams)
    if kind in ("extreme", "extreme_rand"):
        # footprints at the limits of the tile machinery: a few Gaussians
        # covering most of the view (rectangles of hundreds of tiles), thin
        # rotated needles (ellipse-tile decisions far from the bounding box,
        # close to tile corners), and many sub-pixel ones (dilation-dominated)
        big = scenes.uniform_gaussians(rng, 12, log_scale_mu=-1.0, log_scale_sigma=0.3, extent=0.6)
        needle = scenes.uniform_gaussians(rng, 60, log_scale_mu=-5.5, log_scale_sigma=0.3)
        needle[3] = rng.normal(-2.0, 0.3, size=60).astype(np.float32)  # one long axis
        tiny = scenes.uniform_gaussians(rng, 900, log_scale_mu=-7.0, log_scale_sigma=0.5)
        P = np.concatenate([big, needle, tiny], axis=1)
        P[10, :12] = -1.5  # the large ones semi-transparent
        cams = scenes.make_cameras([(0.2, 0.3, 3.0)], [(331, 245)])
        # smooth target: the loss gradient keeps its sign over large areas;
        # uniform random target: it flips from pixel to pixel, so the big
        # Gaussians' sums over ~10^4 pixels cancel to far below their terms
        if kind == "extreme":
            return P, 0, cams, scenes.smooth_target(rng, cams, 8)
        return P, 0, cams, scenes.uniform_target(rng, cams)
    if kind == "ortho":
        P = scenes.uniform_gaussians(rng, 800, log_scale_mu=-2.8)
        cams = scenes.make_cameras([(0.0, 1.0, 4.0)], [(72, 72)], model=1, ortho_scale=24.0)
        return P, 0, cams, scenes.uniform_target(rng, cams)
    raise KeyError(kind)
