"""Pins of the oracle's eigen-decomposition (App. A.3), Steepest Density
Control (Theorem 2, Algorithm 1) and instance sort."""
import json
import os

import numpy as np
import pytest
from scipy.special import expit

from paper_2505_05587_amd import scenes
from tests.helpers import tiny_scene

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_eigh_closed_form_cases(oracle):
    cases = json.load(open(os.path.join(GOLDEN, "eigen_closed_form.json")))["cases"]
    for c in cases:
        A = np.array(c["A"], np.float64)
        lam, vec = oracle.eigh(A[None])
        np.testing.assert_allclose(lam[0], c["eigenvalues"], atol=1e-13)
        if "v_min" in c:
            np.testing.assert_allclose(vec[0][:, 0], c["v_min"], atol=1e-13)


def test_eigh_matches_lapack_on_random_symmetric(oracle):
    rng = np.random.default_rng(50)
    B = rng.normal(size=(10000, 3, 3)) * np.exp(rng.normal(0, 3, size=(10000, 1, 1)))
    S = B + np.swapaxes(B, 1, 2)
    lam, vec = oracle.eigh(S)
    ref = np.linalg.eigvalsh(S)
    scale = np.abs(ref).max(axis=1, keepdims=True)
    assert (np.abs(lam - ref) <= 1e-13 * scale).all()
    # residual and orthonormality of the eigenvector columns
    res = np.einsum("kij,kjl->kil", S, vec) - vec * lam[:, None, :]
    assert (np.linalg.norm(res, axis=1) <= 1e-12 * scale).all()
    np.testing.assert_allclose(np.einsum("kji,kjl->kil", vec, vec), np.broadcast_to(np.eye(3), S.shape), atol=1e-12)
    # canonical sign: the largest-magnitude component of v_min is positive
    v = vec[:, :, 0]
    assert (v[np.arange(len(v)), np.abs(v).argmax(axis=1)] > 0).all()


def test_smith_trigonometric_roots_agree(oracle):
    # App. A.3: A = p B + q I, q = tr(A)/3, p = sqrt(tr((A - qI)^2)/6),
    # beta = 2 cos(acos(det(B)/2)/3 + 2 k pi / 3); the smallest root is k = 1.
    rng = np.random.default_rng(51)
    B0 = rng.normal(size=(2000, 3, 3))
    S = B0 + np.swapaxes(B0, 1, 2)
    lam, _ = oracle.eigh(S)
    q = np.trace(S, axis1=1, axis2=2) / 3
    Aq = S - q[:, None, None] * np.eye(3)
    p = np.sqrt(np.einsum("kij,kji->k", Aq, Aq) / 6)
    detB = np.linalg.det(Aq / p[:, None, None])
    phi = np.arccos(np.clip(detB / 2, -1, 1)) / 3
    roots = np.stack([q + 2 * p * np.cos(phi + 2 * k * np.pi / 3) for k in range(3)], 1)
    np.testing.assert_allclose(np.sort(roots, 1), lam, atol=1e-9 * np.abs(lam).max())
    np.testing.assert_allclose(roots[:, 1], lam[:, 0], atol=1e-9 * np.abs(lam).max())


def _random_S(rng, n):
    B = rng.normal(size=(n, 3, 3))
    S = B + np.swapaxes(B, 1, 2)
    S[: n // 4] = np.einsum("kij,kjl->kil", B[: n // 4], np.swapaxes(B[: n // 4], 1, 2))  # PSD: no split
    return S


def test_densify_rule_and_layout(oracle):
    # Theorem 2 / Algorithm 1: split iff lambda_min < eps_split into
    # (p + eps v_min, o/2) and (p - eps v_min, o/2); others untouched.
    rng = np.random.default_rng(52)
    n = 500
    P = scenes.clustered_gaussians(rng, n, 20, sh_degree=1)
    S = _random_S(rng, n)
    S9 = S.reshape(n, 9).T.copy()
    eps, eps_split = 0.01, -1e-6
    out = oracle.densify(P, 1, S9, 1.0, eps, eps_split)
    lam, vec = oracle.eigh(S)
    np.testing.assert_allclose(out["lambda_min"], lam[:, 0])
    split = lam[:, 0] < eps_split
    np.testing.assert_array_equal(out["split"], split)
    assert out["n_out"] == n + split.sum()
    assert split[: n // 4].sum() == 0 and split.sum() > n // 2
    Q = out["params"]
    o = 0
    for i in range(n):
        if not split[i]:
            np.testing.assert_array_equal(Q[:, o], P[:, i].astype(np.float64))
            o += 1
            continue
        a, b = Q[:, o], Q[:, o + 1]
        p = P[0:3, i].astype(np.float64)
        np.testing.assert_allclose(0.5 * (a[0:3] + b[0:3]), p, rtol=1e-15, atol=1e-15)
        np.testing.assert_allclose(0.5 * (a[0:3] - b[0:3]), eps * vec[i][:, 0], rtol=1e-12, atol=1e-15)
        for c in (a, b):
            assert expit(c[10]) == pytest.approx(0.5 * expit(np.float64(P[10, i])), rel=1e-13)
            np.testing.assert_array_equal(c[3:10], P[3:10, i].astype(np.float64))
            np.testing.assert_array_equal(c[11:], P[11:, i].astype(np.float64))
        o += 2
    assert o == out["n_out"]


def test_densify_scale_and_threshold(oracle):
    # S is averaged over the interval before the test (Algorithm 1); a positive
    # scale does not change the split set at eps_split = 0, the threshold does
    rng = np.random.default_rng(53)
    n = 300
    P = scenes.uniform_gaussians(rng, n)
    S9 = _random_S(rng, n).reshape(n, 9).T.copy()
    a = oracle.densify(P, 0, S9, 1.0, 0.01, 0.0)
    b = oracle.densify(P, 0, S9, 1.0 / 100.0, 0.01, 0.0)
    np.testing.assert_array_equal(a["split"], b["split"])
    np.testing.assert_allclose(b["lambda_min"], a["lambda_min"] / 100.0, rtol=1e-12, atol=1e-15)
    c = oracle.densify(P, 0, S9, 1.0, 0.01, -1e9)
    assert c["n_out"] == n and not c["split"].any()
    small = oracle.densify(P, 0, S9, 1.0, 0.01, 0.0, out_cap=n)
    assert small["n_out"] == -1 and small["needed"] == a["n_out"]


def test_densify_increment_budget(oracle):
    # Variants, increment budget: with more candidates than the budget K, the
    # K smallest lambda_min split (Theorem 2: the loss decrease of a split is
    # lambda_min / 2); equal lambda_min: lower index first.  Eigenvalues from
    # LAPACK, selection from numpy's stable argsort.
    rng = np.random.default_rng(54)
    n = 400
    P = scenes.uniform_gaussians(rng, n)
    S = _random_S(rng, n)
    S[300:310] = S[200]  # ties with one another
    S9 = S.reshape(n, 9).T.copy()
    lam = np.linalg.eigvalsh(S)[:, 0]
    cand = np.nonzero(lam < -1e-6)[0]
    assert len(cand) > 150
    for K in (1, 17, 150, len(cand), len(cand) + 5):
        out = oracle.densify(P, 0, S9, 1.0, 0.01, -1e-6, budget=K)
        keep = cand[np.argsort(lam[cand], kind="stable")][:K]
        want = np.zeros(n, bool)
        want[keep] = True
        if K < len(cand):
            kth = np.sort(lam[cand])[K - 1]
            near = np.abs(lam - kth) < 1e-12 * np.abs(S).max()
            np.testing.assert_array_equal(out["split"][~near], want[~near])
            assert out["split"].sum() == K
        else:
            np.testing.assert_array_equal(out["split"], want)
        assert out["n_out"] == n + out["split"].sum()
    # exact ties: the budget boundary inside the tied group keeps the lowest indices
    tied = [200] + list(range(300, 310))
    K = int(np.sum(lam[cand] < lam[200])) + 4
    out = oracle.densify(P, 0, S9, 1.0, 0.01, -1e-6, budget=K)
    assert out["split"][[200, 300, 301, 302]].all() and not out["split"][303:310].any()
    assert out["split"][tied].sum() == 4


def test_densify_compactest_gate(oracle):
    # Variants, compactest splitting: split only where |G| <= eps_grad and
    # lambda_min < eps_split; G is the interval-averaged position gradient
    rng = np.random.default_rng(55)
    n = 300
    P = scenes.uniform_gaussians(rng, n)
    S9 = _random_S(rng, n).reshape(n, 9).T.copy()
    G = (rng.normal(size=(3, n)) * np.exp(rng.normal(0, 1, size=n))).astype(np.float32)
    lam = np.linalg.eigvalsh(S9.T.reshape(n, 3, 3))[:, 0]
    gn = np.linalg.norm(G.astype(np.float64) * 0.25, axis=0)
    for eps_grad in (0.1, 0.5, 2.0):
        out = oracle.densify(P, 0, S9, 1.0, 0.01, -1e-6, G=G, g_scale=0.25, eps_grad=eps_grad)
        np.testing.assert_array_equal(out["split"], (lam < -1e-6) & (gn <= eps_grad))
    off = oracle.densify(P, 0, S9, 1.0, 0.01, -1e-6, G=G, g_scale=0.25, eps_grad=0.0)
    np.testing.assert_array_equal(off["split"], lam < -1e-6)
    both = oracle.densify(P, 0, S9, 1.0, 0.01, -1e-6, G=G, g_scale=0.25, eps_grad=0.5, budget=10)
    gated = np.nonzero((lam < -1e-6) & (gn <= 0.5))[0]
    keep = gated[np.argsort(lam[gated], kind="stable")][:10]
    assert set(np.nonzero(both["split"])[0]) == set(keep)


def test_densify_adc_gate(oracle):
    # ADC-style condition on G (the mean of the per-step gradient norms, which
    # the Variants section contrasts with the compactest |mean gradient|):
    # split only where g_scale * Gabs >= adc_tau and lambda_min < eps_split.
    # The expected set comes from LAPACK's eigenvalues and numpy norms.
    rng = np.random.default_rng(56)
    n = 300
    P = scenes.uniform_gaussians(rng, n)
    S9 = _random_S(rng, n).reshape(n, 9).T.copy()
    steps = rng.normal(size=(8, 3, n)) * np.exp(rng.normal(0, 1, size=n))
    Gabs = np.linalg.norm(steps, axis=1).sum(axis=0).astype(np.float32)  # sum over 8 steps of |g_t|
    lam = np.linalg.eigvalsh(S9.T.reshape(n, 3, 3))[:, 0]
    mean_norm = Gabs.astype(np.float64) / 8
    for tau in (0.3, 1.0, 3.0):
        out = oracle.densify(P, 0, S9, 1.0, 0.01, -1e-6, g_scale=1 / 8, Gabs=Gabs, adc_tau=tau)
        np.testing.assert_array_equal(out["split"], (lam < -1e-6) & (mean_norm >= tau))
        assert out["split"].sum() < (lam < -1e-6).sum()  # the gate removes some candidates
    off = oracle.densify(P, 0, S9, 1.0, 0.01, -1e-6, g_scale=1 / 8, Gabs=Gabs, adc_tau=0.0)
    np.testing.assert_array_equal(off["split"], lam < -1e-6)
    # the two gates together: mean norm large, norm of the mean small
    G = steps.sum(axis=0).astype(np.float32)
    gn = np.linalg.norm(G.astype(np.float64) / 8, axis=0)
    both = oracle.densify(P, 0, S9, 1.0, 0.01, -1e-6, G=G, g_scale=1 / 8, eps_grad=1.0, Gabs=Gabs, adc_tau=1.0)
    np.testing.assert_array_equal(both["split"], (lam < -1e-6) & (gn <= 1.0) & (mean_norm >= 1.0))


def test_instance_sort_properties(oracle):
    # view-dependent depth sort per tile (Sec. 3, Rasterization): keys are
    # tile | depth, non-decreasing; each visible record appears once per
    # footprint tile (its count, inside its rectangle); ranges partition the
    # list; and the list is numpy's stable sort of the keys in emission order
    # (view, Gaussian, row-major tile).
    P, cams, _ = tiny_scene(54, 300, 64, sh_degree=0)
    cams = scenes.make_cameras([(0, 0, 3.0), (1.5, 0.5, 2.5)], [(64, 48), (40, 72)])
    opts = scenes.opts("3dgs")
    keys, vals, ranges = oracle.sort(P, 0, cams, opts)
    pr = oracle.project(P, 0, cams, opts)
    n = P.shape[1]
    tile = (keys >> np.uint64(32)).astype(np.int64)
    assert (np.diff(keys.astype(np.uint64)) >= 0).all()
    assert len(keys) == int(pr["tiles"].sum())
    np.testing.assert_array_equal(np.bincount(vals, minlength=cams.V * n), pr["tiles"])
    txs = (cams.width.astype(np.int64) + 15) // 16
    tys = (cams.height.astype(np.int64) + 15) // 16
    toff = np.concatenate([[0], np.cumsum(txs * tys)[:-1]])
    v = vals // n
    lt = tile - toff[v]
    x, y = lt % txs[v], lt // txs[v]
    rect = pr["rect"][vals]
    assert ((rect[:, 0] <= x) & (x <= rect[:, 2]) & (rect[:, 1] <= y) & (y <= rect[:, 3])).all()
    np.testing.assert_array_equal(keys & np.uint64(0xFFFFFFFF), pr["depth_bits"][vals])
    em = np.lexsort((tile, vals))  # emission order
    order = np.argsort(keys[em], kind="stable")
    np.testing.assert_array_equal(keys[em][order], keys)
    np.testing.assert_array_equal(vals[em][order], vals)
    covered = np.zeros(len(keys), np.int64)
    for t in range(int((txs * tys).sum())):
        b, e = ranges[t]
        assert (tile[b:e] == t).all()
        covered[b:e] += 1
    assert (covered == 1).all()


def test_paper_constants_fixture():
    c = json.load(open(os.path.join(GOLDEN, "paper_constants.json")))
    assert c["eps_split"]["value"] == -1e-6
    assert c["offspring_weight"]["value"] == 0.5 and c["offspring_count"]["value"] == 2


def test_adam_reference_against_torch_and_first_step(oracle):
    # the oracle's Adam against torch.optim.Adam (a separate implementation,
    # float64 on the CPU), and the textbook first step: |update| = lr where
    # |g| >> eps
    import torch
    rng = np.random.default_rng(56)
    F, n = 23, 40
    lr6 = (1.6e-4, 5e-3, 1e-3, 2.5e-2, 2.5e-3, 1.25e-4)
    p0 = rng.normal(size=(F, n))
    p, m, v = p0.copy(), np.zeros((F, n)), np.zeros((F, n))
    lr_rows = oracle._lr_rows(F, lr6)
    # one torch optimizer per parameter row, each with that row's learning rate
    opts = [torch.optim.Adam([torch.nn.Parameter(torch.tensor(p0[r], dtype=torch.float64))], lr=float(lr_rows[r]),
                             betas=(0.9, 0.999), eps=1e-15) for r in range(F)]
    rows = [o.param_groups[0]["params"][0] for o in opts]
    for t in range(1, 6):
        g = rng.normal(size=(F, n)) * np.exp(rng.normal(0, 2, size=(F, 1)))
        p, m, v = oracle.adam_step(p, g, m, v, t, lr6)
        for r in range(F):
            rows[r].grad = torch.tensor(g[r], dtype=torch.float64)
            opts[r].step()
        ref = np.stack([x.detach().numpy() for x in rows])
        np.testing.assert_allclose(p, ref, rtol=1e-12, atol=1e-15)
        if t == 1:
            np.testing.assert_allclose(np.abs(p - p0), np.broadcast_to(lr_rows[:, None], p.shape), rtol=1e-9)


def test_split_remap_layout(oracle):
    rng = np.random.default_rng(57)
    n = 50
    state = rng.normal(size=(4, n))
    split = rng.random(n) < 0.3
    out = oracle.split_remap(state, split)
    assert out.shape == (4, n + split.sum())
    o = 0
    for i in range(n):
        if split[i]:
            assert (out[:, o] == 0).all() and (out[:, o + 1] == 0).all()
            o += 2
        else:
            np.testing.assert_array_equal(out[:, o], state[:, i])
            o += 1
