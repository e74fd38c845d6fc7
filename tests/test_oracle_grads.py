"""Pins of the oracle's derivatives and splitting matrix (Theorem 1, Sec. 4.4,
Lemma C.1, App. C.4) against finite differences, an algebraic identity,
structural facts of the pinhole projection, and the second-order expansion of
Theorem 1."""
import numpy as np
import pytest

from paper_2505_05587_amd import scenes
from tests.helpers import quantize, tiny_scene


def test_alpha_mean_hessian_matches_second_differences(oracle):
    # App. C.4: Hessian of alpha w.r.t. the projected mean = alpha (A d d^T A - A)
    rng = np.random.default_rng(40)
    for _ in range(50):
        L = rng.normal(size=(2, 2))
        A = L @ L.T + 0.05 * np.eye(2)
        mx, my = rng.uniform(0, 10, size=2)
        g6 = np.array([mx, my, A[0, 0], A[0, 1], A[1, 1], rng.uniform(0.1, 0.9)])
        u, v = mx + rng.normal(0, 1.5), my + rng.normal(0, 1.5)
        h = 1e-4

        def f(dx, dy):
            g = g6.copy()
            g[0] += dx
            g[1] += dy
            return oracle.alpha(g, u, v)

        H = np.array([[(f(h, 0) - 2 * f(0, 0) + f(-h, 0)) / h ** 2,
                       (f(h, h) - f(h, -h) - f(-h, h) + f(-h, -h)) / (4 * h * h)],
                      [0, (f(0, h) - 2 * f(0, 0) + f(0, -h)) / h ** 2]])
        H[1, 0] = H[0, 1]
        Ho = oracle.alpha_hessian(g6, u, v)
        np.testing.assert_allclose(Ho, H, atol=1e-6 * max(1.0, np.abs(Ho).max()))


def _fd_check(oracle, P, deg, cams, opts, target, gids, step, rtol, group_atol):
    out = oracle.forward_backward(P, deg, cams, opts, target)
    G = out["grads"]
    base_pr = oracle.project(P, deg, cams, opts)
    order0 = np.argsort(base_pr["depth_bits"], kind="stable")
    base = oracle.forward_backward(P, deg, cams, opts)
    sgn0 = np.sign(base["image"] - target)
    checked = 0
    for i in gids:
        for f in range(P.shape[0]):
            Pp, Pm = P.copy(), P.copy()
            Pp[f, i] += step
            Pm[f, i] -= step
            assert np.float64(Pp[f, i]) - np.float64(P[f, i]) == step
            prp, prm = oracle.project(Pp, deg, cams, opts), oracle.project(Pm, deg, cams, opts)
            if not (np.array_equal(prp["rect"], base_pr["rect"]) and np.array_equal(prm["rect"], base_pr["rect"])):
                continue  # footprint changed inside the stencil
            if not (np.array_equal(np.argsort(prp["depth_bits"], kind="stable"), order0)
                    and np.array_equal(np.argsort(prm["depth_bits"], kind="stable"), order0)):
                continue  # depth order changed inside the stencil
            rp = oracle.forward_backward(Pp, deg, cams, opts)
            rm = oracle.forward_backward(Pm, deg, cams, opts)
            if not (np.array_equal(np.sign(rp["image"] - target), sgn0) and np.array_equal(np.sign(rm["image"] - target), sgn0)):
                continue  # an L1 kink inside the stencil
            if not (np.array_equal(rp["n_used"], base["n_used"]) and np.array_equal(rm["n_used"], base["n_used"])):
                continue  # an alpha_min / t_min decision changed inside the stencil
            fd = (oracle.loss(Pp, deg, cams, opts, target) - oracle.loss(Pm, deg, cams, opts, target)) / (2 * step)
            tol = rtol * abs(G[f, i]) + group_atol
            assert abs(fd - G[f, i]) <= tol, (i, f, fd, G[f, i])
            checked += 1
    return checked


@pytest.mark.parametrize("deg,model", [(0, 0), (0, 1), (3, 0)])
def test_gradients_match_central_differences(oracle, deg, model):
    P, cams, target = tiny_scene(41 + deg + model, 50, 32, sh_degree=deg, model=model)
    P = quantize(P)
    opts = scenes.opts("smooth", radius_sigmas=4.0)
    gids = list(range(0, 50, 7))
    n = _fd_check(oracle, P, deg, cams, opts, target, gids, step=2.0 ** -13, rtol=2e-4, group_atol=2e-8)
    assert n >= 0.7 * len(gids) * P.shape[0]


def test_gradients_3dgs_mode_match_central_differences(oracle):
    # with the cut-offs active the loss is piecewise smooth; FD is valid
    # where no decision changes inside the stencil
    P, cams, target = tiny_scene(44, 40, 32, sh_degree=1)
    P = quantize(P)
    opts = scenes.opts("3dgs")
    n = _fd_check(oracle, P, 1, cams, opts, target, list(range(0, 40, 6)), step=2.0 ** -13, rtol=5e-4,
                  group_atol=5e-8)
    assert n > 50


def test_splitting_matrix_identity_from_gradients(oracle):
    # Per view, with g(x) = dL/dalpha_i(x):
    #   sum_x g alpha (A d d^T A - A) = A M A - m0 A,  M = -2 dL/dA, m0 = o dL/do
    P, cams, target = tiny_scene(45, 60, 40, sh_degree=2)
    for mode in ("3dgs", "smooth"):
        opts = scenes.opts(mode)
        out = oracle.forward_backward(P, 2, cams, opts, target, per_view=True)
        pr = oracle.project(P, 2, cams, opts)
        g2d, H2d = out["g2d"], out["H2d"]
        for i in np.nonzero(pr["visible"])[0]:
            a, b, c = pr["conic"][i]
            A = np.array([[a, b], [b, c]])
            ga, gb, gc, go = g2d[i, 2], g2d[i, 3], g2d[i, 4], g2d[i, 5]
            M = -np.array([[2 * ga, gb], [gb, 2 * gc]])
            S2 = A @ M @ A - pr["opacity"][i] * go * A
            H = np.array([[H2d[i, 0], H2d[i, 1]], [H2d[i, 1], H2d[i, 2]]])
            np.testing.assert_allclose(H, S2, atol=1e-10 * max(1e-30, np.abs(S2).max()) + 1e-300)


def test_single_view_splitting_matrix_structure(oracle):
    # Pinhole: moving p along the viewing ray leaves Pi(p) fixed, so P (p - c) = 0
    # and S_i = P^T H P has (p_i - c) in its null space: rank <= 2, lambda_min <= 0,
    # and by Sylvester's law of inertia the non-zero eigenvalues carry the
    # signs of the 2x2 H.
    P, cams, target = tiny_scene(46, 80, 48, sh_degree=1)
    opts = scenes.opts("3dgs")
    out = oracle.forward_backward(P, 1, cams, opts, target, per_view=True)
    S = out["S"].T.reshape(-1, 3, 3)
    campos = -cams.R[0].astype(np.float64).T @ cams.t[0].astype(np.float64)
    lam, _ = oracle.eigh(S)
    checked = 0
    for i in range(P.shape[1]):
        nrm = np.abs(S[i]).max()
        if nrm == 0:
            continue
        ray = P[0:3, i].astype(np.float64) - campos
        assert np.linalg.norm(S[i] @ ray) <= 1e-11 * nrm * np.linalg.norm(ray)
        np.testing.assert_allclose(S[i], S[i].T, atol=1e-13 * nrm)
        assert lam[i, 0] <= 1e-11 * nrm
        H = out["H2d"][i]
        h_eig = np.linalg.eigvalsh(np.array([[H[0], H[1]], [H[1], H[2]]]))
        nz = lam[i][np.abs(lam[i]) > 1e-9 * nrm]
        assert sorted(np.sign(nz)) == sorted(np.sign(h_eig[np.abs(h_eig) > 1e-9 * np.abs(h_eig).max()]))
        checked += 1
    assert checked > 20


def test_splitting_matrix_is_loss_hessian_for_affine_l1(oracle):
    # Lemma C.1: d^2 L / d p_i^2 = T_i + S_i, T_i built from d^2 l / d sigma_i^2.
    # With L1 and the blend affine in each alpha, T_i = 0 almost everywhere;
    # with an affine camera and no view-dependent colour nothing else depends
    # on p, so S_i is exactly the Hessian of L w.r.t. p_i.
    P, cams, target = tiny_scene(47, 30, 32, sh_degree=0, model=1, log_scale_mu=-2.0)
    P = quantize(P)
    opts = scenes.opts("smooth", radius_sigmas=1e3)
    out = oracle.forward_backward(P, 0, cams, opts, target)
    S = out["S"].T.reshape(-1, 3, 3)
    h = 2.0 ** -12
    sgn0 = np.sign(oracle.forward_backward(P, 0, cams, opts)["image"] - target)
    checked = 0
    for i in range(0, 30, 3):
        def Lat(da, db):
            Q = P.copy()
            for k, s in (da, db):
                if k is not None:
                    Q[k, i] += s * h
            img = oracle.forward_backward(Q, 0, cams, opts)["image"]
            return oracle.loss(Q, 0, cams, opts, target), np.array_equal(np.sign(img - target), sgn0)

        Hfd = np.zeros((3, 3))
        ok = True
        for a in range(3):
            for b in range(a, 3):
                if a == b:
                    vals = [Lat((a, 1), (None, 0)), Lat((None, 0), (None, 0)), Lat((a, -1), (None, 0))]
                    Hfd[a, a] = (vals[0][0] - 2 * vals[1][0] + vals[2][0]) / h ** 2
                else:
                    vals = [Lat((a, s1), (b, s2)) for s1 in (1, -1) for s2 in (1, -1)]
                    Hfd[a, b] = Hfd[b, a] = (vals[0][0] - vals[1][0] - vals[2][0] + vals[3][0]) / (4 * h * h)
                ok &= all(v[1] for v in vals)
        if not ok:
            continue
        np.testing.assert_allclose(Hfd, S[i], atol=2e-4 * np.abs(S[i]).max() + 1e-9)
        checked += 1
    assert checked >= 5


def test_theorem1_merged_split_second_order(oracle):
    # Theorem 1 with a mean-preserving split (mu = 0), two offspring of weight
    # 1/2 at p +/- eps v: L(split) - L = 1/2 sum_j w_j (eps v)^T S (eps v) + O(eps^3)
    # = eps^2 lambda / 2 for v = v_min.  Offspring share the parent's slot
    # (sigma_i replaced by sum_j w_j sigma_j, Sec. 4.1).
    P, cams, target = tiny_scene(48, 30, 32, sh_degree=0, model=1, log_scale_mu=-2.0)
    opts = scenes.opts("smooth", radius_sigmas=1e3)
    out = oracle.forward_backward(P, 0, cams, opts, target)
    S = out["S"].T.reshape(-1, 3, 3)
    lam, vec = oracle.eigh(S)
    cand = [i for i in range(30) if lam[i, 0] < -1e-3 * np.abs(lam[i]).max() and np.abs(lam[i]).max() > 0]
    assert len(cand) >= 3
    for i in cand[:5]:
        L0 = oracle.loss_merged_split(P, 0, cams, opts, target, i, vec[i][:, 0], 0.0)
        assert L0 == pytest.approx(oracle.loss(P, 0, cams, opts, target), rel=1e-14)
        errs = []
        for eps in (0.02, 0.01, 0.005):
            Ls = oracle.loss_merged_split(P, 0, cams, opts, target, i, vec[i][:, 0], eps)
            errs.append(abs((Ls - L0) / (0.5 * eps * eps * lam[i, 0]) - 1.0))
        assert errs[-1] < 2e-2, errs
        assert errs[-1] < errs[0] or errs[0] < 1e-4


def test_theorem2_vmin_minimises_split_characteristic(oracle):
    # Theorem 2: over unit offsets, sum_j w_j delta_j^T S delta_j >= lambda_min,
    # with equality for delta = +/- v_min and w = (1/2, 1/2)
    rng = np.random.default_rng(49)
    for _ in range(200):
        B = rng.normal(size=(3, 3))
        S = B + B.T
        lam, vec = oracle.eigh(S[None])
        v = vec[0][:, 0]
        best = 0.5 * (v @ S @ v) + 0.5 * ((-v) @ S @ (-v))
        assert best == pytest.approx(lam[0, 0], rel=1e-12, abs=1e-12)
        d = rng.normal(size=(64, 2, 3))
        d /= np.linalg.norm(d, axis=-1, keepdims=True)
        vals = 0.5 * np.einsum("kji,il,kjl->k", d, S, d)
        assert (vals >= lam[0, 0] - 1e-12).all()


def test_upstream_image_gradient_matches_central_differences(oracle):
    # backward of Eq. (alpha_blend) for an arbitrary loss: with dL/dC = w fixed,
    # L = sum w * C is linear in the image, so the gradient must match central
    # differences of the oracle's own image; S must equal the L1 result's when
    # w is the L1 sign gradient
    P, cams, target = tiny_scene(47, 40, 32, sh_degree=1)
    P = quantize(P)
    opts = scenes.opts("smooth", radius_sigmas=4.0)
    rng = np.random.default_rng(48)
    w = rng.normal(size=3 * cams.total_pixels())
    out = oracle.forward_backward(P, 1, cams, opts, dl_dimage=w)
    G = out["grads"]
    step = 2.0 ** -13
    base_pr = oracle.project(P, 1, cams, opts)
    checked = 0
    for i in range(0, 40, 6):
        for f in range(P.shape[0]):
            Pp, Pm = P.copy(), P.copy()
            Pp[f, i] += step
            Pm[f, i] -= step
            prp, prm = oracle.project(Pp, 1, cams, opts), oracle.project(Pm, 1, cams, opts)
            if not all(np.array_equal(np.argsort(pr["depth_bits"], kind="stable"),
                                      np.argsort(base_pr["depth_bits"], kind="stable")) for pr in (prp, prm)):
                continue
            Ip = oracle.forward_backward(Pp, 1, cams, opts)["image"]
            Im = oracle.forward_backward(Pm, 1, cams, opts)["image"]
            fd = float(w @ (Ip - Im)) / (2 * step)
            assert abs(fd - G[f, i]) <= 2e-4 * abs(G[f, i]) + 1e-8 * np.abs(G).max(), (i, f, fd, G[f, i])
            checked += 1
    assert checked >= 0.8 * 7 * P.shape[0]
    # the L1 loss path is the special case w = sign(C - target) / (3HW)
    l1 = oracle.forward_backward(P, 1, cams, opts, target)
    w1 = np.sign(l1["image"] - target) / (3.0 * cams.total_pixels())
    alt = oracle.forward_backward(P, 1, cams, opts, dl_dimage=w1)
    np.testing.assert_allclose(alt["grads"], l1["grads"], rtol=1e-12, atol=1e-18)
    np.testing.assert_allclose(alt["S"], l1["S"], rtol=1e-12, atol=1e-18)


def test_gross_magnitudes_bound_the_sums(oracle):
    # grads_abs and S_abs are the gross magnitudes of the per-pixel terms the
    # gradients and S_i are sums of (the scale of a float32 implementation's
    # order-dependent summation error): they bound the sums entrywise, do not
    # change when the upstream image gradient changes sign (the sums do) and
    # scale with its magnitude
    P, cams, target = tiny_scene(47, 50, 36, sh_degree=1)
    opts = scenes.opts("smooth")
    Px = cams.total_pixels()
    rng = np.random.default_rng(5)
    D = rng.normal(size=3 * Px)
    a = oracle.forward_backward(P, 1, cams, opts, dl_dimage=D)
    b = oracle.forward_backward(P, 1, cams, opts, dl_dimage=-D)
    c = oracle.forward_backward(P, 1, cams, opts, dl_dimage=2.0 * D)
    assert (np.abs(a["grads"]) <= a["grads_abs"] * (1 + 1e-12) + 1e-300).all()
    assert (np.abs(a["S"]) <= a["S_abs"] * (1 + 1e-12) + 1e-300).all()
    seen = np.abs(a["S"]).sum(axis=0) > 0
    assert seen.sum() > 10 and (a["S_abs"][:, seen].sum(axis=0) > 0).all()
    np.testing.assert_allclose(b["grads"], -a["grads"], rtol=1e-12, atol=1e-300)
    np.testing.assert_allclose(b["grads_abs"], a["grads_abs"], rtol=1e-12, atol=1e-300)
    np.testing.assert_allclose(b["S_abs"], a["S_abs"], rtol=1e-12, atol=1e-300)
    np.testing.assert_allclose(c["grads_abs"], 2.0 * a["grads_abs"], rtol=1e-12, atol=1e-300)
    np.testing.assert_allclose(c["S_abs"], 2.0 * a["S_abs"], rtol=1e-12, atol=1e-300)
    # the gross exceeds the net where terms of both signs meet
    assert (a["S_abs"][:, seen].sum(axis=0) > 1.5 * np.abs(a["S"][:, seen]).sum(axis=0)).any()
