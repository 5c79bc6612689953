"""Training-side quantities next to the renderer (Sec. 4.2, "Implementation
and Optimization"), float64, written from their definitions.

* Densification statistic: with no screen-space mean available, the
  gradient of each splat's mean is used, scaled by half its distance to the
  camera in view space. Per view v the loss L_v contributes
  |dL_v/dmu| * |mu - c_v| / 2 to the Gaussian's running sum, and the view
  counts towards its number of views when the Gaussian is visible there
  (its screen box of Sec. 3.2 holds a pixel centre).
* Opacity decay: during densification every opacity is multiplied by
  lambda_o (0.9995); in logit space x' = logit(lambda_o sigmoid(x)).
"""
from __future__ import annotations

import numpy as np
import torch

from . import bins, render, splat

F64 = torch.float64


def view_visible(means, log_scales, quats, opacity_logits, cam, settings):
    """[n] bool: the Gaussian survives culling and its screen box holds at
    least one pixel centre of the view."""
    prep = splat.prepare(means, log_scales, quats, opacity_logits, cam, settings.tau_alpha)
    _, ok, _ = bins.pixel_rects(prep, cam)
    return ok


def mean_grad_stat(params, sh_degree, cams, settings, weights):
    """Sums over the views of |dL_v/dmu| |mu - c_v| / 2, with
    L_v = sum(weights[v] * C_v), and the per-Gaussian count of views in
    which it is visible. params: float64-castable arrays (means, log-scales,
    quaternions, opacity logits, SH)."""
    n = np.asarray(params[0]).shape[0]
    stat = np.zeros(n)
    count = np.zeros(n)
    for cam, G in zip(cams, weights):
        ps = [torch.tensor(np.asarray(a), dtype=F64) for a in params]
        mu = ps[0].clone().requires_grad_(True)
        img = render.render(mu, *ps[1:], sh_degree, cam, settings, cull=False)
        (img * torch.as_tensor(G, dtype=F64)).sum().backward()
        g = mu.grad.numpy()
        dist = np.linalg.norm(np.asarray(params[0], np.float64) - cam.center[None, :], axis=1)
        stat += np.linalg.norm(g, axis=1) * dist / 2.0
        count += view_visible(*params[:4], cam, settings)
    return stat, count


def opacity_decay(logits, lam=0.9995):
    """logit(lam * sigmoid(x)), float64."""
    x = torch.as_tensor(np.asarray(logits), dtype=F64)
    o = torch.sigmoid(x) * lam
    return (torch.log(o) - torch.log1p(-o)).numpy()
