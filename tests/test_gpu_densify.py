"""GPU parity of the split-selection variants (the paper's "Variants"
section): the increment budget (the K candidates with the smallest
lambda_min, ties by index), the compactest gate (|G| <= eps_grad) and the
ADC-style gate (mean per-step gradient norm >= adc_tau)."""
import numpy as np
import pytest
import torch

from paper_2505_05587_amd import pipeline, scenes

pytestmark = pytest.mark.gpu


def _problem(seed, n):
    rng = np.random.default_rng(seed)
    P = scenes.clustered_gaussians(rng, n, 100, sh_degree=1)
    B = rng.normal(size=(n, 3, 3)) * np.exp(rng.normal(0, 1, size=(n, 1, 1)))
    S = B + np.swapaxes(B, 1, 2)
    S[: n // 5] = np.einsum("kij,kjl->kil", B[: n // 5], np.swapaxes(B[: n // 5], 1, 2))
    S[n // 2: n // 2 + 40] = S[n // 3]  # exact ties
    S = S.astype(np.float32)
    S6 = np.stack([S[:, 0, 0], S[:, 0, 1], S[:, 0, 2], S[:, 1, 1], S[:, 1, 2], S[:, 2, 2]]).astype(np.float32)
    G = (rng.normal(size=(3, n)) * np.exp(rng.normal(0, 1, size=n))).astype(np.float32)
    return P, S.reshape(n, 9).T.astype(np.float64), np.ascontiguousarray(S6), G


def _key(lam32):
    b = lam32.astype(np.float32).view(np.uint32).astype(np.uint64)
    return np.where(b & 0x80000000, (~b) & 0xFFFFFFFF, b | 0x80000000)


def _gpu(P, S6, **kw):
    dev = torch.device("cuda", 0)
    G = kw.pop("G", None)
    Gabs = kw.pop("Gabs", None)
    out = pipeline.densify(torch.from_numpy(P).to(dev), 1, torch.from_numpy(S6).to(dev), 1.0, 0.01, -1e-6,
                           G=None if G is None else torch.from_numpy(G).to(dev),
                           Gabs=None if Gabs is None else torch.from_numpy(Gabs).to(dev), **kw)
    torch.cuda.synchronize()
    return dict(split=out["split"].cpu().numpy().astype(bool), lam=out["lambda_min"].cpu().numpy(),
                n_out=out["n_out"], params=None if out["params"] is None else out["params"].cpu().numpy())


@pytest.mark.parametrize("budget", [1, 37, 1000, 10 ** 6])
def test_increment_budget(oracle, budget):
    n = 20000
    P, S9, S6, _ = _problem(60, n)
    print(f"\n[case] densify budget={budget}", flush=True)
    free = _gpu(P, S6)
    got = _gpu(P, S6, budget=budget)
    cand = np.nonzero(free["split"])[0]
    # exact rule on the GPU's own float32 lambda_min: smallest keys, ties by index
    order = cand[np.lexsort((cand, _key(free["lam"][cand])))]
    want = np.zeros(n, bool)
    want[order[:budget]] = True
    np.testing.assert_array_equal(got["split"], want)
    assert got["n_out"] == n + min(budget, len(cand))
    # against the oracle where lambda_min is clear of the selection threshold
    ref = oracle.densify(P, 1, S9, 1.0, 0.01, -1e-6, budget=budget)
    Sn = np.linalg.norm(S9, axis=0)
    if budget < len(cand):
        thr = np.sort(ref["lambda_min"][ref["split"]])[-1]
        sure = np.abs(ref["lambda_min"] - thr) > 1e-5 * Sn
    else:
        sure = np.abs(ref["lambda_min"] + 1e-6) > 1e-4 * Sn
    np.testing.assert_array_equal(got["split"][sure], ref["split"][sure])
    # the split rows are the unbudgeted ones, minus the dropped offspring
    if got["params"] is not None and free["params"] is not None:
        assert got["params"].shape[1] == n + got["split"].sum()


def test_compactest_gate_and_budget(oracle):
    n = 20000
    P, S9, S6, G = _problem(61, n)
    print("\n[case] densify compactest gate", flush=True)
    Sn = np.linalg.norm(S9, axis=0)
    for eps_grad, budget in [(0.5, 0), (2.0, 0), (2.0, 500)]:
        got = _gpu(P, S6, G=G, g_scale=0.25, eps_grad=eps_grad, budget=budget)
        ref = oracle.densify(P, 1, S9, 1.0, 0.01, -1e-6, G=G, g_scale=0.25, eps_grad=eps_grad, budget=budget)
        gn = np.linalg.norm(0.25 * G.astype(np.float64), axis=0)
        sure = (np.abs(ref["lambda_min"] + 1e-6) > 1e-4 * Sn) & (np.abs(gn - eps_grad) > 1e-9)
        if budget:
            thr = np.sort(ref["lambda_min"][ref["split"]])[-1]
            sure &= np.abs(ref["lambda_min"] - thr) > 1e-5 * Sn
            assert got["split"].sum() == budget
        np.testing.assert_array_equal(got["split"][sure], ref["split"][sure])
        assert not (got["split"] & (gn > eps_grad * (1 + 1e-6))).any()


def test_adc_gate_with_compactest_and_budget(oracle):
    n = 20000
    P, S9, S6, G = _problem(62, n)
    rng = np.random.default_rng(63)
    Gabs = (np.linalg.norm(G, axis=0) * (1 + rng.random(n) * 3)).astype(np.float32)  # |mean| <= mean |.|
    print("\n[case] densify ADC gate", flush=True)
    Sn = np.linalg.norm(S9, axis=0)
    mean_norm = 0.25 * Gabs.astype(np.float64)
    gn = np.linalg.norm(0.25 * G.astype(np.float64), axis=0)
    for tau, eps_grad, budget in [(0.5, 0.0, 0), (1.5, 0.0, 0), (0.5, 2.0, 0), (0.5, 2.0, 300)]:
        got = _gpu(P, S6, G=G if eps_grad else None, Gabs=Gabs, g_scale=0.25, eps_grad=eps_grad, adc_tau=tau,
                   budget=budget)
        ref = oracle.densify(P, 1, S9, 1.0, 0.01, -1e-6, G=G if eps_grad else None, g_scale=0.25,
                             eps_grad=eps_grad, Gabs=Gabs, adc_tau=tau, budget=budget)
        sure = (np.abs(ref["lambda_min"] + 1e-6) > 1e-4 * Sn) & (np.abs(mean_norm - tau) > 1e-9)
        if eps_grad:
            sure &= np.abs(gn - eps_grad) > 1e-9
        if budget:
            thr = np.sort(ref["lambda_min"][ref["split"]])[-1]
            sure &= np.abs(ref["lambda_min"] - thr) > 1e-5 * Sn
            assert got["split"].sum() == budget
        np.testing.assert_array_equal(got["split"][sure], ref["split"][sure])
        assert not (got["split"] & (mean_norm < tau * (1 - 1e-6))).any()
        assert 0 < ref["split"].sum() < (ref["lambda_min"] < -1e-6).sum()
