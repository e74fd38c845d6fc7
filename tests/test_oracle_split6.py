"""Pins of the oracle's splitting matrix over theta = (p, log-scales), the
widening of dim Theta beyond the position (Sec. 4.4 defines S_i for the
parameters the Hessian is taken over; the paper's experiments use p only).

* alpha as a function of theta (projection maps frozen at the point): at a
  moved log-scale it equals the alpha of the full projection re-run with that
  scale (the covariance map does not depend on s), and at a moved position it
  follows the mean along the exact Jacobian (checked against the projection
  re-run at the moved position to first order);
* its Hessian (second-order forward mode) against central second differences;
* the position block of S over theta equals the dim-3 S, computed by the
  independent mean-Hessian path and the dual-number Jacobian;
* the 6x6 eigensolver against LAPACK, and the dim-6 split layout.
"""
import numpy as np
import pytest

from paper_2505_05587_amd import scenes

pytestmark = pytest.mark.filterwarnings("ignore")


def _scene():
    rng = np.random.default_rng(71)
    P = scenes.uniform_gaussians(rng, 40, log_scale_mu=-2.2, log_scale_sigma=0.4, extent=0.6)
    cams = scenes.make_cameras([(0.3, 0.2, 3.0)], [(48, 40)])
    return P, cams, scenes.uniform_target(rng, cams)


def _visible(oracle, P, cams, opts):
    p = oracle.project(P, 0, cams, opts)
    return p, np.nonzero(p["tiles"] > 0)[0]


def test_alpha_theta6_against_the_projection(oracle):
    P, cams, _ = _scene()
    opts = scenes.opts("smooth")
    p, vis = _visible(oracle, P, cams, opts)
    for i in vis[:8]:
        u, v = float(np.round(p["mean"][i, 0])) + 1.0, float(np.round(p["mean"][i, 1]))
        # log-scale moves: the full projection with the new scale gives the same conic
        ds = np.array([0.05, -0.03, 0.02])
        Q = P.copy()
        Q[3:6, i] = (P[3:6, i].astype(np.float64) + ds).astype(np.float32)
        ds32 = Q[3:6, i].astype(np.float64) - P[3:6, i].astype(np.float64)  # the float32 step actually taken
        q = oracle.project(Q, 0, cams, opts)
        m, A, o = q["mean"][i], q["conic"][i], q["opacity"][i]
        d = np.array([u - m[0], v - m[1]])
        want = o * np.exp(-0.5 * (A[0] * d[0] ** 2 + 2 * A[1] * d[0] * d[1] + A[2] * d[1] ** 2))
        got = oracle.alpha_theta6(P, 0, cams, opts, i, u, v, np.r_[0.0, 0.0, 0.0, ds32])
        assert abs(got - want) <= 1e-12 * max(1.0, abs(want))
        # position moves: the frozen map follows the projection re-run at
        # p + dp up to a second-order remainder (halving dp quarters it)
        a0 = oracle.alpha_theta6(P, 0, cams, opts, i, u, v, np.zeros(6))
        A = p["conic"][i]
        errs = []
        for scale in (0.25, 0.125):
            dp = scale * np.array([2e-3, -4e-3, 3e-3])
            Q = P.copy()
            Q[0:3, i] = (P[0:3, i].astype(np.float64) + dp).astype(np.float32)
            dp32 = Q[0:3, i].astype(np.float64) - P[0:3, i].astype(np.float64)
            m_true = oracle.project(Q, 0, cams, opts)["mean"][i]
            got = oracle.alpha_theta6(P, 0, cams, opts, i, u, v, np.r_[dp32, 0.0, 0.0, 0.0])
            d = np.array([u - m_true[0], v - m_true[1]])
            want = p["opacity"][i] * np.exp(-0.5 * (A[0] * d[0] ** 2 + 2 * A[1] * d[0] * d[1] + A[2] * d[1] ** 2))
            assert abs(got - a0) > 0
            errs.append(abs(got - want))
            assert errs[-1] <= 1e-2 * abs(got - a0)
        assert errs[1] <= 0.35 * errs[0] + 1e-15


def test_hessian_theta6_against_second_differences(oracle):
    P, cams, _ = _scene()
    opts = scenes.opts("smooth")
    p, vis = _visible(oracle, P, cams, opts)
    h = np.array([2e-4, 2e-4, 2e-4, 2e-3, 2e-3, 2e-3])  # position (world units), log-scales
    for i in vis[:6]:
        for du in (0.0, 1.5):
            u, v = float(p["mean"][i, 0]) + du, float(p["mean"][i, 1]) - 0.7
            _, H = oracle.alpha_theta6(P, 0, cams, opts, i, u, v, np.zeros(6), hessian=True)
            f = lambda d: oracle.alpha_theta6(P, 0, cams, opts, i, u, v, d)
            fd = np.zeros((6, 6))
            for a in range(6):
                for b in range(6):
                    ea, eb = np.eye(6)[a] * h[a], np.eye(6)[b] * h[b]
                    fd[a, b] = (f(ea + eb) - f(ea - eb) - f(-ea + eb) + f(-ea - eb)) / (4 * h[a] * h[b])
            Hm = np.zeros((6, 6))
            k = 0
            for a in range(6):
                for b in range(a, 6):
                    Hm[a, b] = Hm[b, a] = H[k]
                    k += 1
            np.testing.assert_allclose(Hm, fd, rtol=2e-4, atol=2e-5 * np.abs(Hm).max())


def test_position_block_equals_dim3_S(oracle):
    P, cams, target = _scene()
    for mode in ("smooth", "3dgs"):
        opts = scenes.opts(mode)
        S21 = oracle.split6(P, 0, cams, opts, target)
        ref = oracle.forward_backward(P, 0, cams, opts, target)["S"]  # [9][n] row-major 3x3
        M6 = oracle.h6_to_mats(S21)
        M3 = ref.T.reshape(-1, 3, 3)
        scale = np.abs(M3).max()
        np.testing.assert_allclose(M6[:, :3, :3], M3, rtol=1e-9, atol=1e-12 * scale)
        assert np.abs(M6[:, 3:, 3:]).max() > 0 and np.abs(M6[:, :3, 3:]).max() > 0


def test_eigh6_against_lapack(oracle):
    rng = np.random.default_rng(72)
    B = rng.normal(size=(500, 6, 6)) * np.exp(rng.normal(0, 1, size=(500, 1, 1)))
    S = B + np.swapaxes(B, 1, 2)
    lam, vec = oracle.eigh_n(S)
    ref = np.linalg.eigvalsh(S)
    err = np.abs(lam - ref) / np.abs(ref).max(axis=1, keepdims=True)
    assert err.max() <= 1e-12, err.max()
    res = np.einsum("kij,kj->ki", S, vec[:, :, 0]) - lam[:, :1] * vec[:, :, 0]
    assert np.abs(res).max() <= 1e-11 * np.abs(ref).max()
    assert np.allclose(np.linalg.norm(vec[:, :, 0], axis=1), 1.0)
    # closed forms: diagonal and a rank-one matrix
    D = np.diag([3.0, -1.0, 2.0, 0.5, -4.0, 1.0])[None]
    lam, vec = oracle.eigh_n(D)
    np.testing.assert_allclose(lam[0], np.sort(np.diag(D[0])))
    np.testing.assert_allclose(np.abs(vec[0][:, 0]), np.eye(6)[4])
    w = np.array([1.0, -2.0, 0.5, 0.0, 1.0, 3.0])
    lam, _ = oracle.eigh_n(-np.outer(w, w)[None])
    np.testing.assert_allclose(lam[0], [-(w @ w), 0, 0, 0, 0, 0], atol=1e-12 * (w @ w))


def test_densify6_layout(oracle):
    rng = np.random.default_rng(73)
    n = 200
    P = scenes.uniform_gaussians(rng, n)
    B = rng.normal(size=(n, 6, 6))
    S = B + np.swapaxes(B, 1, 2)
    S21 = np.stack([S[:, i, j] for i in range(6) for j in range(i, 6)])
    out = oracle.densify6(P, 0, S21, 0.5, 0.01, -1e-6)
    lam = np.linalg.eigvalsh(0.5 * S)
    np.testing.assert_allclose(out["lambda_min"], lam[:, 0], rtol=0, atol=1e-12 * np.abs(lam).max())
    split = out["split"]
    np.testing.assert_array_equal(split, lam[:, 0] < -1e-6)
    assert out["n_out"] == n + split.sum()
    off = np.concatenate([[0], np.cumsum(1 + split)[:-1]])
    o = out["params"]
    P64 = P.astype(np.float64)
    for i in np.nonzero(split)[0][:20]:
        vm = out["vmin"][:, i]
        np.testing.assert_allclose(np.linalg.norm(vm), 1.0)
        np.testing.assert_allclose(0.5 * S[i] @ vm, out["lambda_min"][i] * vm, atol=1e-10 * np.abs(S[i]).max())
        np.testing.assert_allclose(o[0:6, off[i]], P64[0:6, i] + 0.01 * vm, rtol=0, atol=1e-12)
        np.testing.assert_allclose(o[0:6, off[i] + 1], P64[0:6, i] - 0.01 * vm, rtol=0, atol=1e-12)
        sig = 1 / (1 + np.exp(-P64[10, i]))
        np.testing.assert_allclose(1 / (1 + np.exp(-o[10, off[i]])), sig / 2, rtol=1e-12)
        np.testing.assert_array_equal(o[6:10, off[i]], P64[6:10, i])
        np.testing.assert_array_equal(o[11:, off[i] + 1], P64[11:, i])
    for i in np.nonzero(~split)[0][:20]:
        np.testing.assert_array_equal(o[:, off[i]], P64[:, i])
