"""Seeded synthetic scene generators (inputs only).

This module is shared by the oracle tests and the HIP path. It only draws
inputs -- Gaussian parameters, cameras and target images -- and holds none of
the method's arithmetic (no projection, blending, gradients or splitting).

Parameter layout (planar, float32, shape ``[F, n]``):

    rows 0-2   position p (world units)
    rows 3-5   log-scales (per axis)
    rows 6-9   rotation quaternion (w, x, y, z), not necessarily unit length
    row  10    opacity logit (opacity = sigmoid(logit))
    rows 11..  SH colour coefficients, row 11 + 3*k + ch for basis function k
               (k = l*l + l + m) and colour channel ch

``F = 11 + 3 * (d + 1)**2`` for SH degree ``d``.

Cameras follow the pinhole model with world->camera ``x_c = R x + t``, the
camera looking down +z, x to the right and y down; pixel (u, v) is sampled at
the continuous image point (u, v).  ``model`` 0 is the pinhole camera and 1 an
orthographic (affine) camera ``u = fx * x_c + cx``.

Targets are packed per view as ``[3][H][W]`` planes, views back to back.

Workloads (synthetic stand-ins for the paper's Mip-NeRF 360, Tanks & Temples
and Deep Blending scenes, which are not available):

* ``plain_small``  1,000 Gaussians, means U[-1,1]^3, log-scales N(-3,0.5),
  random unit quaternions, opacity logits N(0,1), SH degree 0 with colour
  U[0,1]; one 64x64 camera at distance 3 looking at the origin, 60 deg fov;
  uniform random target.
* ``single_view``  100,000 Gaussians from 200 isotropic clusters (std 0.1) in
  [-1.5,1.5]^3, log-scales N(-4.5,0.7), SH degree 3 coefficients N(0,0.2); one
  800x800 camera on a radius-4 sphere; smooth target (50 blobs).
* ``batched_16``  1,000,000 Gaussians in 2,000 power-law sized clusters
  (exponent 1.5), log-scales N(-5,1), SH degree 3; 16 cameras on a radius-5
  upper hemisphere with resolutions drawn from {979x546, 1237x822, 1297x840,
  1600x1063}; smooth targets.
* ``gradcheck``  the ``plain_small`` generator with 2,000 Gaussians at 128x128.
* ``autograd_4k``  3,000,000 clustered Gaussians (6,000 clusters), 4 views at
  1920x1080, SH degree 3.
* ``densify_32``  3,000,000 clustered Gaussians, 32 views with resolutions from
  {960x540, 1280x720, 1600x900, 1920x1080}.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

# Value of the degree-0 real spherical harmonic, used only to turn a desired
# base colour into its DC coefficient when drawing inputs.
_SH_Y00 = 0.5 / math.sqrt(math.pi)


def num_params(sh_degree: int) -> int:
    return 11 + 3 * (sh_degree + 1) ** 2


@dataclasses.dataclass
class Cameras:
    R: np.ndarray        # [V,3,3] float32, world->camera rotation
    t: np.ndarray        # [V,3] float32
    fx: np.ndarray       # [V] float32
    fy: np.ndarray
    cx: np.ndarray
    cy: np.ndarray
    width: np.ndarray    # [V] int32
    height: np.ndarray   # [V] int32
    model: np.ndarray    # [V] int32 (0 pinhole, 1 orthographic)

    @property
    def V(self) -> int:
        return int(self.width.shape[0])

    def pixels(self) -> np.ndarray:
        return self.width.astype(np.int64) * self.height.astype(np.int64)

    def pixel_offsets(self) -> np.ndarray:
        px = self.pixels()
        return np.concatenate([[0], np.cumsum(px)[:-1]]).astype(np.int64)

    def total_pixels(self) -> int:
        return int(self.pixels().sum())

    def subset(self, views) -> "Cameras":
        views = np.asarray(views, dtype=np.int64)
        return Cameras(*(getattr(self, f.name)[views].copy() for f in dataclasses.fields(self)))


@dataclasses.dataclass
class Scene:
    name: str
    params: np.ndarray       # [F, n] float32
    sh_degree: int
    cams: Cameras
    target: np.ndarray       # packed [sum_v 3*H_v*W_v] float32

    @property
    def n(self) -> int:
        return int(self.params.shape[1])

    def target_view(self, v: int) -> np.ndarray:
        off = self.cams.pixel_offsets()[v] * 3
        h, w = int(self.cams.height[v]), int(self.cams.width[v])
        return self.target[off: off + 3 * h * w].reshape(3, h, w)


# ----------------------------------------------------------------------------
# cameras


def look_at(campos, target=(0.0, 0.0, 0.0), up=(0.0, 1.0, 0.0)):
    """World->camera (R, t) for a camera at ``campos`` looking at ``target``
    (x right, y down, z forward)."""
    campos = np.asarray(campos, dtype=np.float64)
    f = np.asarray(target, dtype=np.float64) - campos
    f /= np.linalg.norm(f)
    up = np.asarray(up, dtype=np.float64)
    if abs(float(np.dot(f, up))) > 0.999:
        up = np.array([0.0, 0.0, 1.0])
    x = np.cross(f, up)
    x /= np.linalg.norm(x)
    y = np.cross(f, x)
    R = np.stack([x, y, f])
    t = -R @ campos
    return R, t


def make_cameras(positions, sizes, fov_x_deg=60.0, model=0, ortho_scale=None) -> Cameras:
    V = len(positions)
    R = np.zeros((V, 3, 3), np.float32)
    t = np.zeros((V, 3), np.float32)
    fx = np.zeros(V, np.float32)
    W = np.zeros(V, np.int32)
    H = np.zeros(V, np.int32)
    for v, (pos, (w, h)) in enumerate(zip(positions, sizes)):
        Rv, tv = look_at(pos)
        R[v], t[v] = Rv, tv
        W[v], H[v] = w, h
        if model == 0:
            fx[v] = (w / 2.0) / math.tan(math.radians(fov_x_deg) / 2.0)
        else:
            fx[v] = ortho_scale if ortho_scale is not None else w / 4.0
    return Cameras(R=R, t=t, fx=fx.copy(), fy=fx.copy(),
                   cx=(W / 2.0).astype(np.float32), cy=(H / 2.0).astype(np.float32),
                   width=W, height=H, model=np.full(V, model, np.int32))


def sphere_positions(rng, count, radius, upper_only=False):
    out = []
    while len(out) < count:
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        if upper_only and d[1] < 0.0:
            d[1] = -d[1]
        if upper_only and d[1] > 0.98:   # keep clear of the look-at pole
            continue
        out.append(d * radius)
    return out


# ----------------------------------------------------------------------------
# Gaussians


def random_quats(rng, n):
    q = rng.normal(size=(4, n))
    q /= np.linalg.norm(q, axis=0, keepdims=True)
    return q


def uniform_gaussians(rng, n, log_scale_mu=-3.0, log_scale_sigma=0.5, extent=1.0):
    """Means U[-extent, extent]^3, SH degree 0 with base colour U[0,1]."""
    P = np.zeros((num_params(0), n), np.float64)
    P[0:3] = rng.uniform(-extent, extent, size=(3, n))
    P[3:6] = rng.normal(log_scale_mu, log_scale_sigma, size=(3, n))
    P[6:10] = random_quats(rng, n)
    P[10] = rng.normal(0.0, 1.0, size=n)
    rgb = rng.uniform(0.0, 1.0, size=(3, n))
    P[11:14] = (rgb - 0.5) / _SH_Y00
    return P.astype(np.float32)


def powerlaw_sizes(n, n_clusters, exponent):
    w = np.arange(1, n_clusters + 1, dtype=np.float64) ** (-exponent)
    exact = w / w.sum() * n
    base = np.floor(exact).astype(np.int64)
    rem = n - int(base.sum())
    order = np.argsort(-(exact - base), kind="stable")
    base[order[:rem]] += 1
    return base


def clustered_gaussians(rng, n, n_clusters, sh_degree=3, log_scale_mu=-4.5, log_scale_sigma=0.7,
                        cluster_std=0.1, extent=1.5, powerlaw=None, sh_sigma=0.2):
    centres = rng.uniform(-extent, extent, size=(n_clusters, 3))
    if powerlaw is None:
        idx = rng.integers(0, n_clusters, size=n)
    else:
        sizes = powerlaw_sizes(n, n_clusters, powerlaw)
        idx = np.repeat(np.arange(n_clusters), sizes)
        rng.shuffle(idx)
    F = num_params(sh_degree)
    P = np.zeros((F, n), np.float32)
    P[0:3] = (centres[idx] + rng.normal(0.0, cluster_std, size=(n, 3))).T
    P[3:6] = rng.normal(log_scale_mu, log_scale_sigma, size=(3, n))
    P[6:10] = random_quats(rng, n)
    P[10] = rng.normal(0.0, 1.0, size=n)
    P[11:] = rng.normal(0.0, sh_sigma, size=(F - 11, n))
    return P


# ----------------------------------------------------------------------------
# targets


def uniform_target(rng, cams: Cameras):
    return rng.uniform(0.0, 1.0, size=3 * cams.total_pixels()).astype(np.float32)


def smooth_target(rng, cams: Cameras, n_blobs=50):
    """Per view: sum of ``n_blobs`` isotropic 2D Gaussian blobs with centres
    U[0,W]x U[0,H], std U[0.03,0.15]*W pixels and per-channel amplitude
    U[0,1], clipped to [0,1]."""
    out = []
    for v in range(cams.V):
        w, h = int(cams.width[v]), int(cams.height[v])
        img = np.zeros((3, h, w), np.float64)
        xs = np.arange(w, dtype=np.float64)
        ys = np.arange(h, dtype=np.float64)
        for _ in range(n_blobs):
            cx, cy = rng.uniform(0, w), rng.uniform(0, h)
            sd = rng.uniform(0.03, 0.15) * w
            amp = rng.uniform(0.0, 1.0, size=3)
            ex = np.exp(-0.5 * ((xs - cx) / sd) ** 2)
            ey = np.exp(-0.5 * ((ys - cy) / sd) ** 2)
            img += amp[:, None, None] * np.outer(ey, ex)[None]
        out.append(np.clip(img, 0.0, 1.0).astype(np.float32).reshape(-1))
    return np.concatenate(out)


# ----------------------------------------------------------------------------
# workloads

BATCHED_SIZES = [(979, 546), (1237, 822), (1297, 840), (1600, 1063)]
DENSIFY_SIZES = [(960, 540), (1280, 720), (1600, 900), (1920, 1080)]


def plain_small(seed=1, n=1000, size=64, dist=3.0):
    rng = np.random.default_rng(seed)
    params = uniform_gaussians(rng, n)
    cams = make_cameras([(0.0, 0.0, dist)], [(size, size)])
    return Scene("plain_small", params, 0, cams, uniform_target(rng, cams))


def gradcheck(seed=4):
    s = plain_small(seed=seed, n=2000, size=128)
    s.name = "gradcheck"
    return s


def single_view(seed=2, n=100_000, size=(800, 800)):
    rng = np.random.default_rng(seed)
    params = clustered_gaussians(rng, n, 200, sh_degree=3, log_scale_mu=-4.5, log_scale_sigma=0.7)
    cams = make_cameras(sphere_positions(rng, 1, 4.0), [size])
    return Scene("single_view", params, 3, cams, smooth_target(rng, cams))


def clustered_multiview(name, seed, n, n_clusters, n_views, sizes, radius, log_scale_mu=-5.0,
                        log_scale_sigma=1.0, sh_degree=3):
    rng = np.random.default_rng(seed)
    params = clustered_gaussians(rng, n, n_clusters, sh_degree=sh_degree, log_scale_mu=log_scale_mu,
                                 log_scale_sigma=log_scale_sigma, powerlaw=1.5)
    pos = sphere_positions(rng, n_views, radius, upper_only=True)
    res = [sizes[int(i)] for i in rng.integers(0, len(sizes), size=n_views)]
    cams = make_cameras(pos, res)
    return Scene(name, params, sh_degree, cams, smooth_target(rng, cams))


def batched_16(seed=3, n=1_000_000, n_views=16):
    return clustered_multiview("batched_16", seed, n, 2000, n_views, BATCHED_SIZES, 5.0)


def autograd_4k(seed=4, n=3_000_000):
    return clustered_multiview("autograd_4k", seed, n, 6000, 4, [(1920, 1080)], 5.0)


def densify_32(seed=5, n=3_000_000):
    return clustered_multiview("densify_32", seed, n, 6000, 32, DENSIFY_SIZES, 5.0)


WORKLOADS = {
    "plain_small": plain_small,
    "gradcheck": gradcheck,
    "single_view": single_view,
    "batched_16": batched_16,
    "autograd_4k": autograd_4k,
    "densify_32": densify_32,
}


def make(name: str, **kw) -> Scene:
    return WORKLOADS[name](**kw)


# Raster conventions.  "3dgs" follows the cut-offs of the 3D Gaussian
# Splatting rasterizer the paper builds on; "smooth" removes every cut-off
# except the tile footprint, so the image is a smooth function of the
# parameters.
OPTS_3DGS = dict(tile_w=16, tile_h=16, near_z=0.2, radius_sigmas=3.0, dilation=0.3, frustum_guard=1.3,
                 alpha_min=1.0 / 255.0, alpha_max=0.99, t_min=1e-4, bg=(0.0, 0.0, 0.0))
OPTS_SMOOTH = dict(OPTS_3DGS, alpha_min=0.0, alpha_max=1.0, t_min=0.0)


def opts(mode="3dgs", **over):
    """Raster options; real values are rounded to float32 so that a float32
    consumer and a float64 consumer see the same numbers."""
    base = dict(OPTS_3DGS if mode == "3dgs" else OPTS_SMOOTH)
    base.update(over)
    for k, v in list(base.items()):
        if isinstance(v, float):
            base[k] = float(np.float32(v))
    base["bg"] = tuple(float(np.float32(x)) for x in base["bg"])
    return base
