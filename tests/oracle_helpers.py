"""Independent closed forms used to pin the oracle (test code, float64).

Nothing here re-types an oracle formula: rho^2 and depth come from the
inverse covariance and the ray's parametric form, projections from the
pinhole model, blending from the plain depth-sorted alpha-blending sum."""
from __future__ import annotations

import math

import numpy as np

from paper_2410_08129_amd.scenes import Camera, RenderSettings, Scene


def rotation_np(q):
    """Rotation matrix of a unit quaternion via the axis-angle (Rodrigues)
    form, an independent route to the quaternion formula."""
    q = np.asarray(q, np.float64)
    q = q / np.linalg.norm(q)
    w, v = q[0], q[1:]
    s = np.linalg.norm(v)
    if s < 1e-300:
        return np.eye(3)
    axis = v / s
    ang = 2.0 * math.atan2(s, w)
    Kx = np.array([[0, -axis[2], axis[1]], [axis[2], 0, -axis[0]], [-axis[1], axis[0], 0]])
    return np.eye(3) + math.sin(ang) * Kx + (1 - math.cos(ang)) * Kx @ Kx


def quat_mul(a, b):
    w1, x1, y1, z1 = a
    w2, x2, y2, z2 = b
    return np.array([w1 * w2 - x1 * x2 - y1 * y2 - z1 * z2,
                     w1 * x2 + x1 * w2 + y1 * z2 - z1 * y2,
                     w1 * y2 - x1 * z2 + y1 * w2 + z1 * x2,
                     w1 * z2 + x1 * y2 - y1 * x2 + z1 * w2])


def pixel_ray(cam: Camera, xs, ys):
    """World-space origin and direction of the pinhole ray through window
    coordinates (xs, ys); the direction has view-space z = 1."""
    Rc = cam.world_to_cam[:, :3].astype(np.float64)
    t = cam.world_to_cam[:, 3].astype(np.float64)
    Ri = np.linalg.inv(Rc)  # float32 rotations are not exactly orthonormal
    o = -Ri @ t
    v = np.array([(xs - cam.cx) / cam.fx, (ys - cam.cy) / cam.fy, 1.0])
    return o, Ri @ v


def ray_min_mahalanobis(mu, scales, q, o, r):
    """min over t of (o + t r - mu)^T Sigma^-1 (o + t r - mu) and its
    argmin t*, with Sigma = R diag(s^2) R^T (needs every s > 0)."""
    R = rotation_np(q)
    Si = R @ np.diag(1.0 / np.asarray(scales, np.float64) ** 2) @ R.T
    D = o - np.asarray(mu, np.float64)
    a = r @ Si @ r
    b = r @ Si @ D
    c = D @ Si @ D
    return c - b * b / a, -b / a


def ray_plane_rho2(mu, scales, q, o, r, zero_axis):
    """rho^2 of a flat splat (one zero axis) from the ray-plane hit point."""
    R = rotation_np(q)
    n = R[:, zero_axis]
    mu = np.asarray(mu, np.float64)
    th = n @ (mu - o) / (n @ r)
    x = o + th * r - mu
    acc = 0.0
    for k in range(3):
        if k != zero_axis:
            acc += (R[:, k] @ x / scales[k]) ** 2
    return acc


def project(cam: Camera, X):
    """Pinhole projection of world points [n,3] to window coordinates."""
    Rc = cam.world_to_cam[:, :3].astype(np.float64)
    t = cam.world_to_cam[:, 3].astype(np.float64)
    V = X @ Rc.T + t
    return np.stack([cam.fx * V[:, 0] / V[:, 2] + cam.cx,
                     cam.fy * V[:, 1] / V[:, 2] + cam.cy], 1), V[:, 2]


def sorted_blend(alpha, colour, depth, bg):
    """Plain depth-sorted alpha blending (Eq. alpha_blending) plus the
    background behind everything."""
    order = sorted(range(len(alpha)), key=lambda i: (depth[i], i))
    C = np.zeros(3)
    T = 1.0
    for i in order:
        C += alpha[i] * T * np.asarray(colour[i])
        T *= 1.0 - alpha[i]
    return C + T * np.asarray(bg, np.float64)


def simple_camera(width=32, height=32, f=40.0, eye_z=0.0, cx=None, cy=None):
    """Camera at (0, 0, eye_z) looking along +z, identity rotation."""
    w2c = np.zeros((3, 4), np.float32)
    w2c[:, :3] = np.eye(3)
    w2c[2, 3] = -eye_z
    return Camera(w2c, float(f), float(f), float(width / 2 if cx is None else cx),
                  float(height / 2 if cy is None else cy), width, height, 0.2)


def make_scene(means, log_scales, quats, logits, colours=None, sh=None, degree=0):
    n = len(means)
    if sh is None:
        c = np.asarray(colours, np.float64)
        sh = ((c - 0.5) / (0.5 / math.sqrt(math.pi)))[:, None, :]
    return Scene(np.asarray(means, np.float32).reshape(n, 3),
                 np.asarray(log_scales, np.float32).reshape(n, 3),
                 np.asarray(quats, np.float32).reshape(n, 4),
                 np.asarray(logits, np.float32).reshape(n),
                 np.asarray(sh, np.float32), degree)


def tiny_random_scene(n=12, seed=3, spread=0.6, depth=4.0, log_scale=-1.6):
    rng = np.random.default_rng(seed)
    means = np.stack([rng.uniform(-spread, spread, n), rng.uniform(-spread, spread, n),
                      depth + rng.uniform(-1.0, 1.0, n)], 1)
    ls = rng.normal(log_scale, 0.3, (n, 3))
    q = rng.normal(0, 1, (n, 4))
    logit = rng.normal(0.5, 1.0, n)
    col = rng.uniform(0.05, 0.95, (n, 3))
    return make_scene(means, ls, q, logit, col)


def settings(**kw):
    return RenderSettings(**kw)
