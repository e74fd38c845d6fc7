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
               dkeys=ras.dkeys.cpu().numpy().view(np.uint32),
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


def packed_index(cams, pix):
    """[len(pix)][3] indices into the packed image of global pixel ids"""
    offs = np.asarray(cams.pixel_offsets(), np.int64)
    wh = (np.asarray(cams.width, np.int64) * np.asarray(cams.height, np.int64))
    v = np.searchsorted(offs, pix, side="right") - 1
    local = pix - offs[v]
    return 3 * offs[v][:, None] + np.arange(3)[None, :] * wh[v][:, None] + local[:, None]


def resolve_pixels(oracle, P, deg, cams, opts, target, pix, g_image, g_used, dl_dimage=None, with_s6=False):
    """The outcome the GPU took at each of the pixels `pix` whose blend takes a
    decision within float32 reach of its threshold (or whose L1 sign is within
    reach of zero).  The oracle computes every outcome of the pixel; the GPU's
    colour and blended count must match one of them.  Returns the chosen
    outcome per pixel and, per Gaussian, the change of its gradient and S
    terms from the oracle's default outcome (``delta``), the alternatives where
    both outcomes fit the image (``either``), the Gaussians touched by pixels
    with two or more such decisions (``excl``) or an alpha that float32 cannot
    evaluate to the image bar (``soft``), and counts."""
    F = P.shape[0]
    pix = np.asarray(pix, np.int64)
    out = dict(rgb={}, T={}, used={}, delta={}, either={}, excl=set(), soft=set(), excl_pix=set(), soft_pix=set(),
               stats=dict(flagged=len(pix), multi=0, gpu_flipped=0, either=0, valunc=0))
    if len(pix) == 0:
        return out
    e = packed_index(cams, pix)
    n3 = np.full((len(pix), 3), 2)
    D = oracle.pixel_variants(P, deg, cams, opts, target, pix, -np.ones(len(pix), np.int32), n3, dl_dimage=dl_dimage,
                              with_s6=with_s6)
    if dl_dimage is None:
        d32 = g_image[e].astype(np.float32) - np.asarray(target, np.float32)[e]
        sg = np.sign(d32).astype(np.int32)
    else:
        sg = np.zeros((len(pix), 3), np.int32)
    pl, fl, sl, role = [], [], [], []
    for k, p in enumerate(pix):
        nd = int(D["ndec"][k])
        if D["valunc"][k]:
            out["stats"]["valunc"] += 1
            out["soft_pix"].add(int(p))
            out["soft"].update(int(i) for i in D["terms"][k][0])
            continue
        if nd >= 2:
            out["stats"]["multi"] += 1
            out["excl_pix"].add(int(p))
            for f in range(-1, nd):
                pl.append(p)
                fl.append(f)
                sl.append([2, 2, 2])
                role.append((k, "X"))
            continue
        pl += [p]
        fl += [-1]
        sl += [list(sg[k])]
        role += [(k, "A")]
        if nd == 1:
            pl.append(p)
            fl.append(0)
            sl.append(list(sg[k]))
            role.append((k, "B"))
    if not pl:
        return out
    var = oracle.pixel_variants(P, deg, cams, opts, target, np.array(pl), np.array(fl), np.array(sl),
                                dl_dimage=dl_dimage, with_s6=with_s6)
    by = {}
    for j, (k, r) in enumerate(role):
        by.setdefault(k, {}).setdefault(r, []).append(j)
    zero = lambda: [np.zeros(F), np.zeros(9), np.zeros(21)]  # noqa: E731

    def terms_of(v, j, sign, acc):
        gid, gr, Sv, *rest = v["terms"][j]
        for t, i in enumerate(gid):
            a = acc.setdefault(int(i), zero())
            a[0] += sign * gr[t]
            a[1] += sign * Sv[t]
            if rest:
                a[2] += sign * rest[0][t]
        return acc

    for k, p in enumerate(pix):
        rk = by.get(k, {})
        if "X" in rk:
            for j in rk["X"]:
                out["excl"].update(int(i) for i in var["terms"][j][0])
            continue
        if "A" not in rk:
            continue
        got = g_image[e[k]]
        cand = []
        for r in ("A", "B"):
            if r not in rk:
                continue
            j = rk[r][0]
            ok = (np.abs(got - var["rgb"][j]) <= 1e-5 + 1e-4 * np.abs(var["rgb"][j])).all()
            ok &= int(g_used[p]) == int(var["n_used"][j])
            if ok:
                cand.append((r, j))
        if not cand:
            raise AssertionError(f"pixel {p}: the GPU's colour {got} / count {g_used[p]} matches no outcome of its "
                                 "in-band decision: " + ", ".join(f"{r}: {var['rgb'][rk[r][0]]} / "
                                                                  f"{var['n_used'][rk[r][0]]}"
                                                                  for r in ("A", "B") if r in rk))
        r, j = cand[0]
        out["rgb"][int(p)] = var["rgb"][j]
        out["T"][int(p)] = var["T_final"][j]
        out["used"][int(p)] = int(var["n_used"][j])
        if r == "B":
            out["stats"]["gpu_flipped"] += 1
        dg = terms_of(D, k, -1.0, terms_of(var, j, 1.0, {}))
        for i, a in dg.items():
            b = out["delta"].setdefault(i, zero())
            for t in range(3):
                b[t] += a[t]
        if len(cand) == 2:  # both outcomes fit the image: either is a correct gradient
            out["stats"]["either"] += 1
            d2 = terms_of(var, j, -1.0, terms_of(var, cand[1][1], 1.0, {}))
            for i, a in d2.items():
                out["either"].setdefault(i, []).append(tuple(a))
    return out


def checked_reference(oracle, P, deg, cams, opts, g, target=None, dl_dimage=None, with_s6=False):
    """The oracle's reference for one GPU run, with every decision that float32
    can take either way resolved instead of excluded (resolve_pixels): the
    reference takes, at each such pixel, the outcome whose colour and blended
    count the GPU's match.  The loss sign the GPU used is its own float32 sign
    of C - target.  Outcomes the image cannot tell apart (a clamp at alpha ~
    alpha_max changes the gradient, not the colour) are both accepted per
    Gaussian (every combination, up to four such pixels per Gaussian; beyond
    that the Gaussian is left out).  Pixels with two or more such decisions
    are excluded with the Gaussians they touch; pixels whose alpha float32
    cannot evaluate to the image bar (thin footprints seen along their long
    axis, pix_valunc) are checked, and their deviations counted, not failed.

    Returns dict(image, T_final, n_used, grads, S, [S6], pix_excl, gauss_excl,
    gauss_either, pix_soft, gauss_soft, stats)."""
    ref = oracle.forward_backward(P, deg, cams, opts, target, dl_dimage=dl_dimage)
    n = P.shape[1]
    out = dict(image=ref["image"].copy(), T_final=ref["T_final"].copy(), n_used=ref["n_used"].copy(),
               grads=ref["grads"].copy(), S=ref["S"].copy(), loss=ref.get("loss"))
    if with_s6:
        out["S6"] = oracle.split6(P, deg, cams, opts, target, dl_dimage=dl_dimage).copy()
    nd, vu, sa = ref["pix_ndec"], ref["pix_valunc"], ref["pix_signamb"]
    flagged = np.nonzero((nd >= 1) | vu | ((sa > 0) & (dl_dimage is None)))[0]
    res = resolve_pixels(oracle, P, deg, cams, opts, target, flagged, g["image"], g["n_used"], dl_dimage=dl_dimage,
                         with_s6=with_s6)
    for p in res["rgb"]:
        e = packed_index(cams, np.array([p]))[0]
        out["image"][e] = res["rgb"][p]
        out["T_final"][p] = res["T"][p]
        out["n_used"][p] = res["used"][p]
    for i, (dg, dS, dS6) in res["delta"].items():
        out["grads"][:, i] += dg
        out["S"][:, i] += dS
        if with_s6:
            out["S6"][:, i] += dS6
    pix_excl = np.zeros(len(nd), bool)
    pix_excl[list(res["excl_pix"])] = True
    pix_soft = np.zeros(len(nd), bool)
    pix_soft[list(res["soft_pix"])] = True
    gauss_excl = np.zeros(n, bool)
    gauss_excl[list(res["excl"])] = True
    gauss_soft = np.zeros(n, bool)
    gauss_soft[list(res["soft"])] = True
    out.update(pix_excl=pix_excl, gauss_excl=gauss_excl, gauss_either=res["either"], pix_soft=pix_soft & ~pix_excl,
               gauss_soft=gauss_soft & ~gauss_excl, stats=res["stats"])
    return out


def check_against(g, vref, cams, what, grads_key="grads", S_key="S6", rel=1e-3, abs_frac=1e-6):
    """Image, transmittance, blended counts, gradients and S of a GPU run
    against checked_reference at the plain bars.  Pixels and Gaussians of
    pix_soft / gauss_soft may deviate (counted); pix_excl / gauss_excl are
    left out.  Prints and returns the fractions."""
    excl_rgb = expand_pixel_mask(vref["pix_excl"], cams)
    soft_rgb = expand_pixel_mask(vref["pix_soft"], cams)
    ok = image_close(g["image"], vref["image"])
    bad = ~ok & ~excl_rgb
    assert not (bad & ~soft_rgb).any(), f"{what}: {(bad & ~soft_rgb).sum()} image values out of tolerance"
    soft_dev = (bad & soft_rgb).reshape(-1)
    pix_soft_dev = np.zeros(len(vref["pix_excl"]), bool)
    if soft_dev.any():
        idx = np.nonzero(soft_dev)[0]
        for v in range(cams.V):
            o = 3 * cams.pixel_offsets()[v]
            wh = int(cams.width[v] * cams.height[v])
            sel = idx[(idx >= o) & (idx < o + 3 * wh)] - o
            pix_soft_dev[cams.pixel_offsets()[v] + (sel % wh)] = True
    keep_px = ~vref["pix_excl"] & ~vref["pix_soft"]
    okT = np.abs(g["T_final"] - vref["T_final"]) <= 1e-5 + 1e-4 * vref["T_final"]
    assert okT[keep_px].all(), f"{what}: transmittance"
    np.testing.assert_array_equal(g["n_used"][keep_px], vref["n_used"][keep_px])
    n = g[grads_key].shape[1]
    # per Gaussian: the plain bar against the reference, or against the
    # reference with the other outcome of a pixel both outcomes of which fit
    G, R = g[grads_key], vref["grads"]
    S9 = vref["S"]
    excl = vref["gauss_excl"].copy()
    either = vref["gauss_either"]
    for i, alts in either.items():
        if len(alts) > 4:
            excl[i] = True
    fails = _group_fails(G, R, ~excl, rel, abs_frac) | _S_fails(g[S_key], S9, ~excl, rel, abs_frac)
    for i in list(np.nonzero(fails)[0]):
        alts = either.get(int(i), [])
        if not alts or len(alts) > 4:
            continue
        one = np.zeros(n, bool)
        one[i] = True
        # every combination of the pixels' outcomes
        for mask in range(1, 1 << len(alts)):
            R2 = R.copy()
            S2 = S9.copy()
            for b, alt in enumerate(alts):
                if (mask >> b) & 1:
                    R2[:, i] += alt[0]
                    S2[:, i] += alt[1]
            if not (_group_fails(G, R2, one, rel, abs_frac, scale_from=R)[i] or
                    _S_fails(g[S_key], S2, one, rel, abs_frac, scale_from=S9)[i]):
                fails[i] = False
                break
    soft = vref["gauss_soft"]
    hard = fails & ~soft
    assert not hard.any(), (f"{what}: {hard.sum()} Gaussians out of tolerance, e.g. {np.nonzero(hard)[0][:8]}")
    st = dict(vref["stats"], pix_excl=float(vref["pix_excl"].mean()), gauss_excl=float(excl.mean()),
              pix_soft_dev=float(pix_soft_dev.mean()), gauss_soft_dev=float((fails & soft).mean()))
    print(f"[checked] {what}: {st}", flush=True)
    return st


def _group_fails(got, ref, keep, rel, abs_frac, scale_from=None):
    scale = ref if scale_from is None else scale_from
    fails = np.zeros(got.shape[1], bool)
    for name, sl in GROUPS.items():
        dn = np.linalg.norm(got[sl] - ref[sl], axis=0)
        rn = np.linalg.norm(ref[sl], axis=0)
        top = np.linalg.norm(scale[sl], axis=0)
        tol = rel * rn + abs_frac * (top[keep].max() if keep.any() else 0.0)
        fails |= keep & (dn > tol)
    return fails


def _S_fails(S6_gpu, S9_ref, keep, rel, abs_frac, scale_from=None):
    M_g = s6_to_mats(S6_gpu)
    M_r = s6_to_mats(s9_to_s6(S9_ref))
    M_s = M_r if scale_from is None else s6_to_mats(s9_to_s6(scale_from))
    dn = np.linalg.norm((M_g - M_r).reshape(len(M_g), -1), axis=1)
    rn = np.linalg.norm(M_r.reshape(len(M_r), -1), axis=1)
    top = np.linalg.norm(M_s.reshape(len(M_s), -1), axis=1)
    tol = rel * rn + abs_frac * (top[keep].max() if keep.any() else 0.0)
    return keep & (dn > tol)


def _deviations(G, Rg, S6g, S9, keep, k, rel, abs_frac):
    """(name, |d|, |ref|, tol) per parameter group and for S of sampled Gaussian k"""
    out = []
    for name, sl in GROUPS.items():
        rn = np.linalg.norm(Rg[sl, k])
        out.append((name, np.linalg.norm(G[sl, k] - Rg[sl, k]), rn,
                    rel * rn + abs_frac * np.linalg.norm(Rg[sl][:, keep], axis=0).max()))
    M_g = s6_to_mats(S6g)
    M_r = s6_to_mats(s9_to_s6(S9))
    rn = np.linalg.norm(M_r[k])
    out.append(("S", np.linalg.norm(M_g[k] - M_r[k]), rn,
                rel * rn + abs_frac * np.linalg.norm(M_r[keep].reshape(int(keep.sum()), -1), axis=1).max()))
    return out


def _fail_detail(G, Rg, S6g, S9, keep, k, rel, abs_frac):
    """|d| / tol per parameter group and for S of sampled Gaussian k"""
    return f"#{k}: " + ", ".join(f"{name} |d|={dn:.3e} |ref|={rn:.3e} tol={tol:.3e}"
                                 for name, dn, rn, tol in _deviations(G, Rg, S6g, S9, keep, k, rel, abs_frac)
                                 if dn > tol)


def sampled_check(oracle, scene, opts, g_image, g_used, grads, S6, gids, what, rel=1e-3, abs_frac=1e-6):
    """Gradients and S of sampled Gaussians of a full-size run against the
    oracle's (every pixel of every tile they touch blended in full), with the
    in-band decisions of those pixels resolved as in checked_reference.
    grads [F][n], S6 [6][n] of the GPU.  Returns the fraction of the sample
    left out (pixels with two or more in-band decisions) and the stats."""
    gids = np.asarray(gids, np.int64)
    g_ref, S_ref, _, flagged = oracle.grads_sampled(scene.params, scene.sh_degree, scene.cams, opts, scene.target,
                                                    gids, flagged=True)
    res = resolve_pixels(oracle, scene.params, scene.sh_degree, scene.cams, opts, scene.target, flagged, g_image,
                         g_used)
    pos = {int(i): k for k, i in enumerate(gids)}
    for i, (dg, dS, _) in res["delta"].items():
        if i in pos:
            g_ref[pos[i]] += dg
            S_ref[pos[i]] += dS
    excl = np.array([int(i) in res["excl"] for i in gids])
    soft = np.array([int(i) in res["soft"] for i in gids]) & ~excl
    G = grads[:, gids]
    Rg = g_ref.T.copy()
    S9 = S_ref.T.copy()
    keep = ~excl
    fails = _group_fails(G, Rg, keep, rel, abs_frac) | _S_fails(S6[:, gids], S9, keep, rel, abs_frac)
    for k in list(np.nonzero(fails)[0]):
        alts = res["either"].get(int(gids[k]), [])
        if not alts or len(alts) > 4:
            continue
        one = np.zeros(len(gids), bool)
        one[k] = True
        for mask in range(1, 1 << len(alts)):
            R2, S2 = Rg.copy(), S9.copy()
            for b, alt in enumerate(alts):
                if (mask >> b) & 1:
                    R2[:, k] += alt[0]
                    S2[:, k] += alt[1]
            if not (_group_fails(G, R2, one, rel, abs_frac, scale_from=Rg)[k] or
                    _S_fails(S6[:, gids], S2, one, rel, abs_frac, scale_from=S9)[k]):
                fails[k] = False
                break
    hard = fails & ~soft
    assert not hard.any(), (f"{what}: sampled Gaussians {gids[hard]} out of tolerance: "
                            + "; ".join(_fail_detail(G, Rg, S6[:, gids], S9, keep, k, rel, abs_frac)
                                        for k in np.nonzero(hard)[0][:4]))
    # the largest |d| / tol of the Gaussians whose deviation is left unchecked
    # (pixels whose alpha float32 cannot evaluate to the image bar)
    soft_worst = max([max(dn / tol for _, dn, _, tol in _deviations(G, Rg, S6[:, gids], S9, keep, k, rel, abs_frac))
                      for k in np.nonzero(fails & soft)[0]], default=0.0)
    st = dict(res["stats"], sampled=len(gids), excluded=float(excl.mean()), soft_dev=float((fails & soft).mean()),
              soft_worst=round(float(soft_worst), 2), flagged_pixels=len(flagged))
    print(f"[sampled] {what}: {st}", flush=True)
    return st


def sample_gaussians(oracle, scene, opts, rng, heavy_tiles=4, per_tile=4, needles=8, random=48, max_tiles=400):
    """Gaussians to check at full size: members of the longest tile lists,
    the most elongated footprints (largest condition number of the projected
    covariance over the views), and random visible ones, all with at most
    `max_tiles` tiles over all views (the oracle blends every pixel of them)"""
    pr = oracle.project(scene.params, scene.sh_degree, scene.cams, opts)
    V, n = scene.cams.V, scene.n
    tiles = pr["tiles"].reshape(V, n).astype(np.int64)
    tot = tiles.sum(0)
    ok = (tot > 0) & (tot <= max_tiles)
    a, b, c = pr["conic"][:, 0], pr["conic"][:, 1], pr["conic"][:, 2]
    hi = 0.5 * (a + c) + np.sqrt(0.25 * (a - c) ** 2 + b * b)
    lo = (a * c - b * b) / np.where(hi > 0, hi, 1.0)
    kappa = np.where(pr["visible"] & (lo > 0), hi / np.where(lo > 0, lo, 1.0), 0.0).reshape(V, n).max(0)
    picks = []
    ln = np.zeros(1, np.int64)
    if heavy_tiles > 0:
        _, vals, ranges = oracle.sort(scene.params, scene.sh_degree, scene.cams, opts)
        ln = ranges[:, 1].astype(np.int64) - ranges[:, 0].astype(np.int64)
    for t in np.argsort(-ln)[:heavy_tiles]:
        ids = np.unique(vals[ranges[t, 0]:ranges[t, 1]].astype(np.int64) % n)
        ids = ids[ok[ids]]
        picks += list(rng.choice(ids, size=min(per_tile, len(ids)), replace=False))
    picks += list(np.argsort(-np.where(ok, kappa, 0.0))[:needles])
    pool = np.setdiff1d(np.nonzero(ok)[0], picks)
    picks += list(rng.choice(pool, size=min(random, len(pool)), replace=False))
    return np.unique(np.asarray(picks, np.int64)), dict(heavy_tile_lengths=ln[np.argsort(-ln)[:heavy_tiles]].tolist(),
                                                         max_kappa=float(kappa[ok].max()))
