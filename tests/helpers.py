"""Small scene builders shared by the tests (inputs only)."""
import numpy as np

from paper_2505_05587_amd import scenes


def pack_params(means, log_scales, quats, logits, sh, sh_degree):
    n = len(means)
    F = scenes.num_params(sh_degree)
    P = np.zeros((F, n), np.float32)
    P[0:3] = np.asarray(means, np.float64).T
    P[3:6] = np.asarray(log_scales, np.float64).T
    P[6:10] = np.asarray(quats, np.float64).T
    P[10] = np.asarray(logits, np.float64)
    P[11:] = np.asarray(sh, np.float64).reshape(n, -1).T
    return P


def ortho_camera(size=32, scale=None, pos=(0.0, 0.0, 5.0)):
    return scenes.make_cameras([pos], [(size, size)], model=1, ortho_scale=scale)


def pinhole_camera(size=32, pos=(0.0, 0.0, 3.0)):
    return scenes.make_cameras([pos], [(size, size)])


def quantize(P, step=2.0 ** -10):
    """Round parameters to a grid so that +/- a power-of-two step stays exact in float32."""
    return (np.round(P.astype(np.float64) / step) * step).astype(np.float32)


def tiny_scene(seed, n, size, sh_degree=0, model=0, log_scale_mu=-2.5, extent=0.8):
    rng = np.random.default_rng(seed)
    if sh_degree == 0:
        P = scenes.uniform_gaussians(rng, n, log_scale_mu=log_scale_mu, log_scale_sigma=0.3, extent=extent)
    else:
        P = scenes.clustered_gaussians(rng, n, max(1, n // 10), sh_degree=sh_degree, log_scale_mu=log_scale_mu,
                                       log_scale_sigma=0.3, cluster_std=0.3, extent=extent * 0.5)
    if model == 0:
        cams = pinhole_camera(size)
    else:
        cams = ortho_camera(size, scale=size / 3.0)
    target = scenes.uniform_target(rng, cams)
    return P, cams, target
