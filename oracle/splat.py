"""Per-Gaussian geometry in float64 (paper Sec. 3.1 and Sec. 3.2).

Follows: the scene representation of Sec. 3.1 (sigmoid opacity, log-space
scales, normalised quaternion); the splat-to-world matrix T and the screen
transform T' = V P M T of Eq. (T_matrix); the opacity-aware cutoff
rho_c = 2 ln(o / tau_alpha) and the inversion-free dual-quadric bounding box
(s, f, p_i, h_i) of Sec. 3.2.

Two input options of Sec. 4.2 and the frame-rate appendix:
  * the 3D smoothing filter (Mip-Splatting, used by the paper in place of a
    screen-space filter): each Gaussian's covariance gets a per-Gaussian
    isotropic variance f added, Sigma' = Sigma + f I, and its peak opacity
    is scaled so that the filtered density is the convolution of the
    unfiltered one with a normalised isotropic Gaussian of variance f:
    o' = o sqrt(det Sigma / det Sigma'). With Sigma = R diag(s^2) R^T this
    is s'_i = sqrt(s_i^2 + f) along the same axes and o' = o prod s_i/s'_i;
  * "baked" inputs: the activations already applied, so the arrays hold
    the scales, unit quaternions and opacities themselves.
"""
from __future__ import annotations

import torch

F64 = torch.float64


def as_f64(x):
    if isinstance(x, torch.Tensor):
        return x.to(F64)
    return torch.as_tensor(x, dtype=F64)


def quat_to_rotation(q):
    """Rotation matrix of the normalised quaternion q = (w, x, y, z).

    The columns of the result are the splat's tangential axes t_u, t_v, t_w
    (Sec. 3.1). Standard unit-quaternion formula."""
    q = q / torch.linalg.norm(q, dim=-1, keepdim=True)
    w, x, y, z = q.unbind(-1)
    R = torch.stack([
        1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y),
        2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x),
        2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y),
    ], dim=-1)
    return R.reshape(q.shape[:-1] + (3, 3))


def activations(log_scales, quats, opacity_logits, filter_var=None, baked=False):
    """s = exp(log-scale) (log-scale -inf gives an exactly zero axis),
    R from the normalised quaternion, o = sigmoid(logit) (Sec. 3.1); baked
    inputs are taken as s, R's quaternion and o directly. With the 3D
    filter's variance f: s' = sqrt(s^2 + f), o' = o prod s / s'."""
    if baked:
        s, o = log_scales, opacity_logits
    else:
        s = torch.exp(log_scales)
        o = torch.sigmoid(opacity_logits)
    R = quat_to_rotation(quats)
    if filter_var is not None:
        f = as_f64(filter_var)
        s_f = torch.sqrt(s * s + f[:, None])
        # a zero axis with no filter variance keeps its opacity factor 1
        ratio = torch.where(s_f > 0, s / torch.where(s_f > 0, s_f, torch.ones_like(s_f)),
                            torch.ones_like(s_f))
        o = o * torch.prod(ratio, dim=1)
        s = s_f
    return s, R, o


def splat_to_world(means, s, R):
    """T of Eq. (T_matrix): columns s_u t_u, s_v t_v, s_w t_w, mu; last row
    (0, 0, 0, 1). Maps normalised splat space (the Gaussian's unit sphere)
    to world space."""
    n = means.shape[0]
    top = torch.cat([R * s[:, None, :], means[:, :, None]], dim=2)  # [n,3,4]
    bottom = torch.tensor([0.0, 0.0, 0.0, 1.0], dtype=F64).expand(n, 1, 4)
    return torch.cat([top, bottom], dim=1)


def camera_matrices(cam, far=1.0e4):
    """Model-view M, projection P (to clip space) and viewport V (to window
    coordinates in pixels) of Sec. 3.2, as 4x4 float64 matrices.

    Camera axes are x right, y down, z forward (OpenCV); P maps view space to
    clip space with w = z and V maps normalised device coordinates [-1, 1]
    to window coordinates [0, W] x [0, H], so that a view point (X, Y, Z)
    lands at window x = fx X / Z + cx, y = fy Y / Z + cy. The depth row is
    a conventional [near, far] mapping; it does not affect x, y."""
    W, H = float(cam.width), float(cam.height)
    fx, fy, cx, cy = (float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy))
    n_, f_ = float(cam.z_near), float(far)
    M = torch.eye(4, dtype=F64)
    M[:3, :] = as_f64(cam.world_to_cam)
    P = torch.tensor([
        [2 * fx / W, 0.0, 2 * cx / W - 1.0, 0.0],
        [0.0, 2 * fy / H, 2 * cy / H - 1.0, 0.0],
        [0.0, 0.0, (f_ + n_) / (f_ - n_), -2 * f_ * n_ / (f_ - n_)],
        [0.0, 0.0, 1.0, 0.0]], dtype=F64)
    V = torch.tensor([
        [W / 2, 0.0, 0.0, W / 2],
        [0.0, H / 2, 0.0, H / 2],
        [0.0, 0.0, 0.5, 0.5],
        [0.0, 0.0, 0.0, 1.0]], dtype=F64)
    return M, P, V


def opacity_cutoff(o, tau_alpha):
    """rho_c = 2 ln(o / tau_alpha): the squared splat-space radius beyond
    which o exp(-rho^2/2) < tau_alpha (Sec. 3.2; rho_c is a squared radius)."""
    return 2.0 * torch.log(o / tau_alpha)


def screen_bbox(Tp, rho_c):
    """Tight screen-space box of the rho_c-ellipsoid without inversion
    (Sec. 3.2, Weyrich et al.'s form of Sigg et al.'s bound):

      s   = <(rc, rc, rc, -1), T'_4 . T'_4>
      f   = (rc, rc, rc, -1) / s
      p_i = <f, T'_i . T'_4>
      h_i = sqrt(p_i^2 - <f, T'_i . T'_i>)

    Returns s [n], p [n,3], h [n,3] for i = 1, 2, 3 (x, y, z). h^2 is clamped
    at 0 against round-off for flat or line-like splats."""
    n = Tp.shape[0]
    w = torch.stack([rho_c, rho_c, rho_c, -torch.ones_like(rho_c)], dim=-1)  # [n,4]
    T4 = Tp[:, 3, :]
    s = (w * T4 * T4).sum(-1)
    f = w / s[:, None]
    p = torch.stack([(f * Tp[:, i, :] * T4).sum(-1) for i in range(3)], dim=-1)
    q = torch.stack([(f * Tp[:, i, :] * Tp[:, i, :]).sum(-1) for i in range(3)], dim=-1)
    h = torch.sqrt(torch.clamp(p * p - q, min=0.0))
    return s, p, h


def prepare(means, log_scales, quats, opacity_logits, cam, tau_alpha, filter_var=None,
            baked=False):
    """Per-Gaussian quantities shared by the renderer and the tile lists.

    Culling (the paper does not spell it out): a Gaussian is dropped when
    o <= tau_alpha (empty cutoff), when its view-space centre depth is at or
    in front of the near plane, or when s >= 0 (its rho_c-ellipsoid reaches
    the camera plane, so no finite screen box exists). A box that is not
    finite in x or y after round-off is treated the same way."""
    means, log_scales = as_f64(means), as_f64(log_scales)
    quats, opacity_logits = as_f64(quats), as_f64(opacity_logits)
    s_ax, R, o = activations(log_scales, quats, opacity_logits, filter_var, baked)
    T = splat_to_world(means, s_ax, R)
    M, P, V = camera_matrices(cam)
    MT = M @ T
    Tp = V @ P @ MT
    rho_c = opacity_cutoff(o, tau_alpha)
    s_q, p, h = screen_bbox(Tp, rho_c)
    z_view = MT[:, 2, 3]
    finite = torch.isfinite(p[:, :2]).all(1) & torch.isfinite(h[:, :2]).all(1)
    visible = (o > tau_alpha) & (z_view > cam.z_near) & (s_q < 0) & finite
    return dict(scales=s_ax, R=R, o=o, T=T, MT=MT, Tp=Tp, rho_c=rho_c,
                s=s_q, p=p, h=h, visible=visible, z_view=z_view)


def mean_view_depth32(means, cam):
    """Sort key of sorted blending: the view depth of each mean, the third
    row of the world-to-camera transform applied to mu in float64 (the
    products of the float32 inputs are exact; the sum is taken x, y, z,
    then the translation), rounded to float32. [n] numpy float32."""
    mu = as_f64(means).detach().numpy()
    w = as_f64(cam.world_to_cam).numpy()
    z = ((w[2, 0] * mu[:, 0] + w[2, 1] * mu[:, 1]) + w[2, 2] * mu[:, 2]) + w[2, 3]
    return z.astype('float32')

