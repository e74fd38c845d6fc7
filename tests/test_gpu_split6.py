"""GPU parity of the splitting matrix over theta = (p, log-scales) (dim 6)
and of the dim-6 Steepest Density Control, against the oracle's
second-order forward-mode Hessian and its 6x6 Jacobi solver."""
import numpy as np
import pytest
import torch

from paper_2505_05587_amd import pipeline, scenes
from tests.gpu_common import check_against, checked_reference, scene_small

pytestmark = pytest.mark.gpu

PAIRS = [(i, j) for i in range(6) for j in range(i, 6)]


def _mats(S21):
    n = S21.shape[1]
    M = np.zeros((n, 6, 6))
    for k, (i, j) in enumerate(PAIRS):
        M[:, i, j] = S21[k]
        M[:, j, i] = S21[k]
    return M


@pytest.mark.parametrize("kind", ["plain_small", "multiview", "ortho", "sh3_pinhole"])
@pytest.mark.parametrize("mode", ["smooth", "3dgs"])
def test_split6_matches_oracle(oracle, kind, mode):
    P, deg, cams, target = scene_small(kind)
    opts = scenes.opts(mode)
    dev = torch.device("cuda", 0)
    print(f"\n[case] split6 kind={kind} mode={mode} n={P.shape[1]} V={cams.V}", flush=True)
    ras = pipeline.Rasterizer(pipeline.CameraBatch(cams, opts, dev), deg, capacity=1024)
    Pt = torch.from_numpy(np.ascontiguousarray(P)).to(dev)
    tg = torch.from_numpy(np.ascontiguousarray(target)).to(dev)
    fs = ras.forward(Pt, tg, count_used=True)
    grads = torch.zeros_like(Pt)
    S3 = torch.zeros((6, P.shape[1]), dtype=torch.float32, device=dev)
    S6 = torch.zeros((21, P.shape[1]), dtype=torch.float32, device=dev)
    ras.backward6(Pt, grads, S6, S=S3, target=tg)
    torch.cuda.synchronize()
    g = dict(image=fs.image.cpu().numpy().astype(np.float64), T_final=fs.T_final.cpu().numpy(),
             n_used=ras.n_used.cpu().numpy(), grads=grads.cpu().numpy().astype(np.float64),
             S6=S3.cpu().numpy().astype(np.float64))
    vref = checked_reference(oracle, P, deg, cams, opts, g, target=target, with_s6=True)
    # the gradients and dim-3 S of the dim-6 backward are those of the plain one
    check_against(g, vref, cams, f"split6 {kind}/{mode}")
    rel = 1e-3
    Mg, Mr = _mats(S6.cpu().numpy().astype(np.float64)), _mats(vref["S6"])
    keep = ~vref["gauss_excl"]
    d = np.linalg.norm((Mg - Mr).reshape(-1, 36), axis=1)
    r = np.linalg.norm(Mr.reshape(-1, 36), axis=1)
    tol = rel * r + 1e-6 * r[keep].max()
    bad = keep & (d > tol)
    for i in np.nonzero(bad)[0]:  # a pixel both of whose outcomes fit the image: either S6 is correct
        alts = vref["gauss_either"].get(int(i), [])
        if len(alts) == 1:
            M2 = _mats(vref["S6"][:, [i]] + alts[0][2][:, None])[0]
            bad[i] = np.linalg.norm(Mg[i] - M2) > rel * np.linalg.norm(M2) + 1e-6 * r[keep].max()
    assert not bad.any(), f"{bad.sum()} of {keep.sum()} S6 out of tolerance; worst {np.max((d / tol)[keep]):.2f}"
    print(f"[bar] split6 {kind}/{mode} S6: worst |d|/tol = {np.max((d / tol)[keep]):.3f}", flush=True)
    # and its position block is the dim-3 S (two fp64 lifts of the same
    # moments: per Gaussian within the bar)
    S3g = S3.cpu().numpy().astype(np.float64)
    M3 = np.zeros((P.shape[1], 3, 3))
    for k, (i, j) in enumerate([(0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2)]):
        M3[:, i, j] = M3[:, j, i] = S3g[k]
    d3 = np.linalg.norm((Mg[:, :3, :3] - M3).reshape(-1, 9), axis=1)
    r3 = np.linalg.norm(M3.reshape(-1, 9), axis=1)
    assert (d3 <= rel * r3 + 1e-6 * r3.max()).all()
    assert np.abs(Mr[keep][:, 3:, 3:]).max() > 0


def test_densify6_matches_oracle(oracle):
    rng = np.random.default_rng(81)
    n = 5000
    P = scenes.clustered_gaussians(rng, n, 60, sh_degree=1)
    B = rng.normal(size=(n, 6, 6)) * np.exp(rng.normal(0, 1, size=(n, 1, 1)))
    S = B + np.swapaxes(B, 1, 2)
    S[: n // 5] = np.einsum("kij,kjl->kil", B[: n // 5], np.swapaxes(B[: n // 5], 1, 2))  # PSD: no split
    S21 = np.stack([S[:, i, j] for i, j in PAIRS]).astype(np.float32)
    dev = torch.device("cuda", 0)
    print("\n[case] densify6", flush=True)
    out = pipeline.densify6(torch.from_numpy(P).to(dev), 1, torch.from_numpy(np.ascontiguousarray(S21)).to(dev),
                            0.5, 0.01, -1e-6)
    torch.cuda.synchronize()
    ref = oracle.densify6(P, 1, S21.astype(np.float64), 0.5, 0.01, -1e-6)
    Sn = 0.5 * np.linalg.norm(S21.astype(np.float64), axis=0) * np.sqrt(2)
    lam = out["lambda_min"].cpu().numpy().astype(np.float64)
    np.testing.assert_allclose(lam, ref["lambda_min"], rtol=0, atol=1e-6 * Sn.max())
    sure = np.abs(ref["lambda_min"] + 1e-6) > 1e-4 * Sn
    split = out["split"].cpu().numpy().astype(bool)
    np.testing.assert_array_equal(split[sure], ref["split"][sure])
    assert out["n_out"] == n + split.sum() and not split[: n // 5].any()
    # eigenvectors where the gap to the next eigenvalue is clear
    vg = out["vmin"].cpu().numpy().astype(np.float64)
    ev = np.linalg.eigvalsh(0.5 * S)
    gap = (ev[:, 1] - ev[:, 0]) > 1e-3 * Sn
    cosang = np.abs(np.sum(vg * ref["vmin"], axis=0))
    assert (cosang[gap] >= 1 - 1e-4).all()
    # offspring: theta +- eps v in position and log-scale rows (an unordered
    # pair: -v is as good an eigenvector), o/2, the rest copied
    params = out["params"].cpu().numpy().astype(np.float64)
    if (split == ref["split"]).all():
        off = np.concatenate([[0], np.cumsum(1 + split)[:-1]])
        idx = np.nonzero(split & gap)[0]
        a, b = params[:, off[idx]], params[:, off[idx] + 1]
        ra, rb = ref["params"][:, off[idx]], ref["params"][:, off[idx] + 1]
        tol = 2e-6 * (1 + np.abs(ra[0:6]))
        same = (np.abs(a[0:6] - ra[0:6]) <= tol).all(axis=0) & (np.abs(b[0:6] - rb[0:6]) <= tol).all(axis=0)
        swap = (np.abs(a[0:6] - rb[0:6]) <= tol).all(axis=0) & (np.abs(b[0:6] - ra[0:6]) <= tol).all(axis=0)
        assert (same | swap).all()
        np.testing.assert_allclose(a[10], ra[10], rtol=1e-5, atol=1e-6)
        np.testing.assert_array_equal(a[6:10], ra[6:10])
        np.testing.assert_array_equal(b[11:], rb[11:])
        keep = np.nonzero(~split)[0]
        np.testing.assert_array_equal(params[:, off[keep]], ref["params"][:, off[keep]])
