"""Pins of the oracle's per-pixel variants (the two outcomes of a cut-off
decision taken within float32 reach of its threshold, Eq. alpha_blend):

- the default variants of all pixels, summed, are the full gradients and S
  of the forward/backward (the per-pixel decomposition of Theorem 1's sum);
- a flipped decision equals a tile-free brute-force blend in plain Python
  with that one decision inverted, for each kind of cut-off: footprint
  radius, alpha_max clamp, alpha_min skip, t_min stop.  The thresholds are
  set within 1e-7 relative of the fp64 value of one (pixel, Gaussian) pair
  so that the decision lies inside its band.
"""
import numpy as np
import pytest

from paper_2505_05587_amd import scenes
from tests.helpers import tiny_scene


def _terms_sum(res, F, n):
    G = np.zeros((F, n))
    S = np.zeros((9, n))
    for gid, gr, Sv in res["terms"]:
        np.add.at(G.T, gid, gr)
        np.add.at(S.T, gid, Sv)
    return G, S


@pytest.mark.parametrize("mode", ["3dgs", "smooth"])
def test_default_variants_sum_to_forward_backward(oracle, mode):
    P, cams, target = tiny_scene(31, 60, 24, log_scale_mu=-2.2)
    opts = scenes.opts(mode, bg=(0.1, 0.2, 0.3))
    ref = oracle.forward_backward(P, 0, cams, opts, target)
    Px = cams.total_pixels()
    pix = np.arange(Px)
    res = oracle.pixel_variants(P, 0, cams, opts, target, pix, -np.ones(Px, np.int32), np.full((Px, 3), 2))
    G, S = _terms_sum(res, P.shape[0], P.shape[1])
    np.testing.assert_allclose(G, ref["grads"], rtol=1e-10, atol=1e-12 * np.abs(ref["grads"]).max())
    np.testing.assert_allclose(S, ref["S"], rtol=1e-10, atol=1e-12 * np.abs(ref["S"]).max())
    img = ref["image"].reshape(3, -1).T
    np.testing.assert_allclose(res["rgb"], img, rtol=1e-14, atol=1e-15)
    np.testing.assert_allclose(res["T_final"], ref["T_final"], rtol=1e-14, atol=1e-300)
    np.testing.assert_array_equal(res["n_used"], ref["n_used"])
    np.testing.assert_array_equal(res["ndec"], ref["pix_ndec"])


def _brute_pixel(pr, opts, n, x, y, force=None):
    """One pixel, every visible Gaussian, ordered by (float32 depth, index),
    composited front to back with the cut-offs; force = (kind, i) inverts that
    one decision of Gaussian i (kind: footprint, alpha_max, alpha_min, t_min)."""
    k2 = opts["radius_sigmas"] ** 2
    fk, fi = force if force else (None, -1)
    cand = []
    for i in range(n):
        if not pr["visible"][i]:
            continue
        (mx, my), (a, b, c) = pr["mean"][i], pr["conic"][i]
        dx, dy = x - mx, y - my
        inside = a * dx * dx + 2 * b * dx * dy + c * dy * dy <= k2
        if fk == "footprint" and fi == i:
            inside = not inside
        if inside:
            cand.append(i)
    cand.sort(key=lambda i: (np.float32(pr["depth"][i]), i))
    T, C, k = 1.0, np.zeros(3), 0
    for i in cand:
        (mx, my), (a, b, c), o = pr["mean"][i], pr["conic"][i], pr["opacity"][i]
        dx, dy = x - mx, y - my
        raw = o * np.exp(-0.5 * (a * dx * dx + 2 * b * dx * dy + c * dy * dy))
        clamp = raw > opts["alpha_max"]
        if fk == "alpha_max" and fi == i:
            clamp = not clamp
        al = opts["alpha_max"] if clamp else raw
        skip = al < opts["alpha_min"]
        if fk == "alpha_min" and fi == i:
            skip = not skip
        if skip:
            continue
        stop = T * (1 - al) < opts["t_min"]
        if fk == "t_min" and fi == i:
            stop = not stop
        if stop:
            break
        C += pr["rgb"][i] * al * T
        T *= 1 - al
        k += 1
    return C + T * np.asarray(opts["bg"]), T, k


def _pair_quantities(pr, opts, n, x, y):
    """(i, q, raw alpha, T in front) of the pixel's blended entries under opts"""
    k2 = opts["radius_sigmas"] ** 2
    cand = []
    for i in range(n):
        if not pr["visible"][i]:
            continue
        (mx, my), (a, b, c) = pr["mean"][i], pr["conic"][i]
        dx, dy = x - mx, y - my
        q = a * dx * dx + 2 * b * dx * dy + c * dy * dy
        if q <= k2:
            cand.append((np.float32(pr["depth"][i]), i, q, pr["opacity"][i] * np.exp(-0.5 * q)))
    cand.sort()
    out, T = [], 1.0
    for _, i, q, raw in cand:
        al = min(opts["alpha_max"], raw)
        if al < opts["alpha_min"]:
            continue
        out.append((i, q, raw, T))
        T *= 1 - al
    return out


@pytest.mark.parametrize("kind", ["footprint", "alpha_max", "alpha_min", "t_min"])
def test_flipped_decision_matches_brute_force(oracle, kind):
    P, cams, target = tiny_scene(32, 50, 24, log_scale_mu=-2.0)
    P[10] = 3.0  # opacities ~0.95: several entries per pixel, transmittance falls fast
    base = scenes.opts("3dgs", bg=(0.1, 0.2, 0.3))
    pr = oracle.project(P, 0, cams, base)
    n = P.shape[1]
    W = int(cams.width[0])
    checked = 0
    for y in range(4, 20, 3):
        for x in range(4, 20, 3):
            ents = _pair_quantities(pr, base, n, x, y)
            if len(ents) < 3:
                continue
            i, q, raw, Tin = ents[1]
            opts = dict(base)
            # the threshold a hair (1e-7 relative, well inside the band) to one
            # side of the pair's value, so that the default outcome is clear
            if kind == "footprint":
                opts["radius_sigmas"] = float(np.sqrt(q) * (1 + 1e-7))      # inside by default
            elif kind == "alpha_max":
                opts["alpha_max"] = float(raw * (1 - 1e-7))                 # clamped by default
            elif kind == "alpha_min":
                opts["alpha_min"] = float(raw * (1 - 1e-7))                 # blended by default
            else:
                opts["t_min"] = float(Tin * (1 - min(base["alpha_max"], raw)) * (1 + 1e-7))  # stops by default
            pid = y * W + x
            dflt = oracle.pixel_variants(P, 0, cams, opts, target, [pid], [-1], [[2, 2, 2]])
            if dflt["ndec"][0] != 1:
                continue  # another decision of this pixel is in its band too
            flip = oracle.pixel_variants(P, 0, cams, opts, target, [pid], [0], [[2, 2, 2]])
            prk = oracle.project(P, 0, cams, opts)
            for res, force in ((dflt, None), (flip, (kind, i))):
                C, T, k = _brute_pixel(prk, opts, n, x, y, force)
                np.testing.assert_allclose(res["rgb"][0], C, rtol=1e-12, atol=1e-14)
                np.testing.assert_allclose(res["T_final"][0], T, rtol=1e-12, atol=1e-300)
                assert res["n_used"][0] == k
            # the two outcomes differ: the decision matters for this pixel (at
            # alpha ~ alpha_max the clamp barely moves the colour and changes
            # the Gaussian's gradient: a clamped alpha is constant)
            if kind == "alpha_max":
                gd, gg = dflt["terms"][0], flip["terms"][0]
                a = gd[1][list(gd[0]).index(i)]
                b = gg[1][list(gg[0]).index(i)]
                assert np.abs(a[:11] - b[:11]).max() > 0
            else:
                assert np.abs(flip["rgb"][0] - dflt["rgb"][0]).max() > 0 or flip["n_used"][0] != dflt["n_used"][0]
            checked += 1
    assert checked >= 3
