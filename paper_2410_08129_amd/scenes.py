"""Seeded synthetic scenes and pinhole cameras.

This module only draws inputs: Gaussian parameter arrays and cameras. It
holds none of the renderer's arithmetic, so the FP64 oracle and the HIP path
both consume exactly the same FP32 values from here.

Every array is generated in float64 with ``numpy.random.default_rng(seed)``
(PCG64) and cast to float32 at the end. The draw order inside a scene is
fixed: centres, cluster ids, offsets, log-scales, quaternions, opacity
logits, SH coefficients, then cameras.

Parameter conventions (Sec. 3.1 of the paper: mean, log-space scales,
quaternion, sigmoid opacity, SH up to degree 3 with 48 coefficients):

* ``means``          [N,3]   world-space centres
* ``log_scales``     [N,3]   s = exp(log_scale); -inf encodes a zero axis
* ``quats``          [N,4]   (w, x, y, z), not normalised
* ``opacity_logits`` [N]     o = sigmoid(logit)
* ``sh``             [N,(deg+1)^2,3]  coefficient index l*l + l + m

Camera conventions: world-to-camera ``[R|t]`` (3x4, row-major), OpenCV axes
(x right, y down, z forward), focal lengths and principal point in pixels,
pixel (i, j) has its centre at (i + 0.5, j + 0.5).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

# Value of the constant real SH basis function 1/(2 sqrt(pi)); used only to
# pick DC coefficients so that the DC colour is uniform in [0, 1].
_Y00 = 0.5 / math.sqrt(math.pi)


@dataclasses.dataclass
class Scene:
    means: np.ndarray
    log_scales: np.ndarray
    quats: np.ndarray
    opacity_logits: np.ndarray
    sh: np.ndarray
    sh_degree: int

    @property
    def n(self) -> int:
        return int(self.means.shape[0])

    def subset(self, idx) -> "Scene":
        idx = np.asarray(idx)
        return Scene(self.means[idx].copy(), self.log_scales[idx].copy(),
                     self.quats[idx].copy(), self.opacity_logits[idx].copy(),
                     self.sh[idx].copy(), self.sh_degree)

    def arrays(self):
        return (self.means, self.log_scales, self.quats, self.opacity_logits, self.sh)


@dataclasses.dataclass
class Camera:
    world_to_cam: np.ndarray  # [3,4] float32
    fx: float
    fy: float
    cx: float
    cy: float
    width: int
    height: int
    z_near: float = 0.2

    def crop(self, x0: int, y0: int, w: int, h: int) -> "Camera":
        """Same camera restricted to the pixel window [x0, x0+w) x [y0, y0+h)."""
        return Camera(self.world_to_cam.copy(), self.fx, self.fy,
                      float(np.float32(self.cx - x0)), float(np.float32(self.cy - y0)),
                      int(w), int(h), self.z_near)

    @property
    def center(self) -> np.ndarray:
        """Camera centre in world space (the point that maps to the view-space
        origin, -R^-1 t), float64."""
        R = self.world_to_cam[:, :3].astype(np.float64)
        t = self.world_to_cam[:, 3].astype(np.float64)
        return -np.linalg.solve(R, t)


@dataclasses.dataclass
class RenderSettings:
    K: int = 8
    tau_alpha: float = 1.0 / 255.0
    tau_core: float = 0.05
    alpha_max: float = 0.99
    bg: tuple = (0.0, 0.0, 0.0)
    tile_w: int = 16
    tile_h: int = 16
    lds_batch: int = 0          # forward records per batch: 0 = tile pixels, 2x allowed at 8x8
    cost_order: bool = False    # rasterize tiles in descending instance-count order
    grad_overwrite: bool = False  # backward writes gradients instead of adding to them
    tile_cull: bool = False     # drop box tiles that the rho_c-ellipse does not reach
    persistent: bool = False    # raster workgroups pull tiles from an atomic queue
    no_tail: bool = False       # inference without the tail (forward only)
    baked: bool = False         # inputs hold scales, unit quaternions and opacities
    sorted_blend: bool = False  # alpha blending in per-tile mean-depth order instead of HT
    tau_T: float = 1.0e-4       # sorted blending stops before transmittance drops below this


def look_at(eye, target, up_world, fov_x_deg, width, height, z_near=0.2) -> Camera:
    """Pinhole camera at ``eye`` looking at ``target``; ``up_world`` is the
    world direction that appears up in the image (camera y points down)."""
    eye = np.asarray(eye, np.float64)
    f = np.asarray(target, np.float64) - eye
    f /= np.linalg.norm(f)
    down = -np.asarray(up_world, np.float64)
    y = down - np.dot(down, f) * f
    y /= np.linalg.norm(y)
    x = np.cross(y, f)
    R = np.stack([x, y, f])
    t = -R @ eye
    fx = (width / 2.0) / math.tan(math.radians(fov_x_deg) / 2.0)
    w2c = np.concatenate([R, t[:, None]], axis=1).astype(np.float32)
    return Camera(w2c, float(np.float32(fx)), float(np.float32(fx)),
                  width / 2.0, height / 2.0, int(width), int(height), z_near)


def _quats(rng, n):
    q = rng.normal(0.0, 1.0, (n, 4))
    return q / np.linalg.norm(q, axis=1, keepdims=True)


def _sh(rng, n, degree, hi_std):
    nb = (degree + 1) ** 2
    sh = np.zeros((n, nb, 3))
    colour = rng.uniform(0.0, 1.0, (n, 3))
    sh[:, 0, :] = (colour - 0.5) / _Y00
    if nb > 1:
        sh[:, 1:, :] = rng.normal(0.0, hi_std, (n, nb - 1, 3))
    return sh


def _pack(means, ls, q, logit, sh, degree) -> Scene:
    f = np.float32
    return Scene(np.ascontiguousarray(means, f), np.ascontiguousarray(ls, f),
                 np.ascontiguousarray(q, f), np.ascontiguousarray(logit, f),
                 np.ascontiguousarray(sh, f), degree)


def uniform_scene(n=4096, seed=0) -> Scene:
    """Small scene: means U[-1,1]^3, log-scales N(-4, 0.5), opacity logits
    N(0, 1), SH degree 0 with DC colour U[0,1]."""
    rng = np.random.default_rng(seed)
    means = rng.uniform(-1.0, 1.0, (n, 3))
    ls = rng.normal(-4.0, 0.5, (n, 3))
    q = _quats(rng, n)
    logit = rng.normal(0.0, 1.0, n)
    sh = _sh(rng, n, 0, 0.0)
    return _pack(means, ls, q, logit, sh, 0)


def clustered_scene(n, n_clusters=64, seed=0, sh_degree=3, degenerate_frac=0.0,
                    near_degenerate_frac=0.0) -> Scene:
    """Mixture of anisotropic clusters: centres U[-10,10]^3, member offsets
    with per-axis standard deviations (2, 0.5, 2), log-scales N(-3.5, 0.7),
    opacity logits N(0, 1.5), SH DC colour U[0,1] and higher bands N(0, 0.05).

    ``degenerate_frac`` of the Gaussians (seeded) get one uniformly chosen
    axis with log-scale -inf (scale exactly 0); a disjoint
    ``near_degenerate_frac`` get one axis with scale 1e-7."""
    rng = np.random.default_rng(seed)
    centres = rng.uniform(-10.0, 10.0, (n_clusters, 3))
    cid = rng.integers(0, n_clusters, n)
    offs = rng.normal(0.0, 1.0, (n, 3)) * np.array([2.0, 0.5, 2.0])
    means = centres[cid] + offs
    ls = rng.normal(-3.5, 0.7, (n, 3))
    q = _quats(rng, n)
    logit = rng.normal(0.0, 1.5, n)
    sh = _sh(rng, n, sh_degree, 0.05)
    if degenerate_frac > 0.0 or near_degenerate_frac > 0.0:
        perm = rng.permutation(n)
        n_deg = int(round(degenerate_frac * n))
        n_near = int(round(near_degenerate_frac * n))
        deg = perm[:n_deg]
        near = perm[n_deg:n_deg + n_near]
        ls[deg, rng.integers(0, 3, n_deg)] = -np.inf
        ls[near, rng.integers(0, 3, n_near)] = math.log(1e-7)
    return _pack(means, ls, q, logit, sh, sh_degree)


def smooth_target(height, width, seed=1) -> np.ndarray:
    """U[0,1] noise at (H/16, W/16, 3), bilinearly upsampled (half-pixel
    centres, edge clamp) to [3, H, W] float32."""
    rng = np.random.default_rng(seed)
    h = max(1, height // 16)
    w = max(1, width // 16)
    lo = rng.uniform(0.0, 1.0, (h, w, 3))

    def axis(n_out, n_in):
        pos = (np.arange(n_out) + 0.5) * (n_in / n_out) - 0.5
        pos = np.clip(pos, 0.0, n_in - 1)
        i0 = np.floor(pos).astype(np.int64)
        i1 = np.minimum(i0 + 1, n_in - 1)
        return i0, i1, pos - i0

    y0, y1, fy = axis(height, h)
    x0, x1, fx = axis(width, w)
    top = lo[y0][:, x0] * (1 - fx)[None, :, None] + lo[y0][:, x1] * fx[None, :, None]
    bot = lo[y1][:, x0] * (1 - fx)[None, :, None] + lo[y1][:, x1] * fx[None, :, None]
    img = top * (1 - fy)[:, None, None] + bot * fy[:, None, None]
    return np.ascontiguousarray(img.transpose(2, 0, 1), np.float32)


# ---------------------------------------------------------------------------
# Workloads. Each returns (scene, cameras, settings).
# ---------------------------------------------------------------------------

def workload_small(seed=0):
    """4,096 uniform Gaussians, 128x128, fov 60 deg, camera 3 units from the
    origin looking at it, K = 4, 16x16 tiles, forward only."""
    scene = uniform_scene(4096, seed)
    cam = look_at((0, 0, -3), (0, 0, 0), (0, -1, 0), 60.0, 128, 128)
    return scene, [cam], RenderSettings(K=4, tile_w=16, tile_h=16)


def workload_1080p(seed=0, n=1_000_000):
    """1M clustered Gaussians (64 clusters), SH degree 3, 1920x1080,
    fov 50 deg, camera at (0,0,-25) looking at the origin, K = 8, 8x8 tiles."""
    scene = clustered_scene(n, 64, seed)
    cam = look_at((0, 0, -25), (0, 0, 0), (0, -1, 0), 50.0, 1920, 1080)
    return scene, [cam], RenderSettings(K=8, tile_w=8, tile_h=8)


def workload_720p(seed=0, n=1_000_000):
    """The 1080p scene seen by a 1280x720 camera (forward + backward)."""
    scene = clustered_scene(n, 64, seed)
    cam = look_at((0, 0, -25), (0, 0, 0), (0, -1, 0), 50.0, 1280, 720)
    return scene, [cam], RenderSettings(K=8, tile_w=8, tile_h=8)


_RESOLUTIONS = ((640, 480), (1280, 720), (1600, 900), (1920, 1080))


def workload_multiview(seed=0, n=3_000_000, n_views=16):
    """3M clustered Gaussians (128 clusters); 16 views of uneven resolution
    on a sphere of radius 25 looking at the origin, fov 50 deg, K = 8."""
    scene = clustered_scene(n, 128, seed)
    rng = np.random.default_rng(seed + 1000)
    cams = []
    for _ in range(n_views):
        w, h = _RESOLUTIONS[int(rng.integers(0, len(_RESOLUTIONS)))]
        e = rng.normal(0.0, 1.0, 3)
        e = 25.0 * e / np.linalg.norm(e)
        up = np.array([0.0, -1.0, 0.0])
        if abs(np.dot(up, -e / np.linalg.norm(e))) > 0.99:
            up = np.array([0.0, 0.0, 1.0])
        cams.append(look_at(e, (0, 0, 0), up, 50.0, w, h))
    return scene, cams, RenderSettings(K=8, tile_w=8, tile_h=8)


def workload_stress(seed=0, n=6_000_000):
    """6M clustered Gaussians with 10% exactly-degenerate and 2%
    near-degenerate splats, SH degree 3, 3840x2160, fov 70 deg, K = 16."""
    scene = clustered_scene(n, 64, seed, 3, 0.10, 0.02)
    cam = look_at((0, 0, -25), (0, 0, 0), (0, -1, 0), 70.0, 3840, 2160)
    return scene, [cam], RenderSettings(K=16, tile_w=8, tile_h=8)


def random_crops(cam: Camera, n, size, seed=0):
    """``n`` seeded crop windows of ``size`` x ``size`` inside ``cam``."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        x0 = int(rng.integers(0, max(1, cam.width - size + 1)))
        y0 = int(rng.integers(0, max(1, cam.height - size + 1)))
        out.append((x0, y0, cam.crop(x0, y0, size, size)))
    return out
