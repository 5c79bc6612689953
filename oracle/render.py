"""Brute-force float64 renderer: every Gaussian at every pixel ray, then the
hybrid-transparency composite (paper Sec. 3.2 and Sec. 3.3).

Steps, in the paper's order:
  1. activations, T, T' = V P M T, rho_c, screen box and culling   (splat.py)
  2. colour from SH at the camera-to-mean direction                 (sh.py)
  3. per pixel: planes -> splat space -> Pluecker d, m -> rho^2, depth (rays.py)
  4. fragment iff the Gaussian is not culled, |d| > 0 and rho^2 <= rho_c;
     alpha = min(alpha_max, o exp(-rho^2 / 2))   (Eq. gauss_alpha_computation)
  5. hybrid-transparency composite                                   (blend.py)
     (or, with settings.sorted_blend, alpha blending in the global order
     of the means' view depths with an early stop: blend.sorted_alpha)

The only thing added for speed is an optional, conservative crop cull that
is independent of the paper's box: a Gaussian is skipped when the sphere of
radius sqrt(rho_c) * max(s) around its mean misses the frustum of the image
window. That sphere contains the rho_c-ellipsoid, so no fragment is lost.
"""
from __future__ import annotations

import dataclasses

import numpy as np
import torch

from . import blend, rays, sh, splat

F64 = torch.float64


@dataclasses.dataclass
class Prepared:
    idx: torch.Tensor        # indices (into the full scene) of the kept Gaussians
    o: torch.Tensor
    rho_c: torch.Tensor
    Tp: torch.Tensor
    MT: torch.Tensor
    colour: torch.Tensor


def _f64(x):
    return splat.as_f64(x)


def frustum_candidates(prep, cam):
    """Conservative sphere-vs-window-frustum test in view space."""
    c = prep['MT'][:, :3, 3]
    r = torch.sqrt(torch.clamp(prep['rho_c'], min=0.0)) * prep['scales'].max(dim=1).values
    fx, fy, cx, cy = float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy)
    W, H = float(cam.width), float(cam.height)
    normals = torch.tensor([[fx, 0.0, cx], [-fx, 0.0, W - cx],
                            [0.0, fy, cy], [0.0, -fy, H - cy]], dtype=F64)
    normals = normals / torch.linalg.norm(normals, dim=1, keepdim=True)
    dist = c @ normals.T                                   # [n,4]
    inside = (dist >= -r[:, None]).all(dim=1)
    return inside & (c[:, 2] + r > cam.z_near)


def prepare(means, log_scales, quats, opacity_logits, sh_coeffs, sh_degree, cam,
            settings, cull=True, filter_var=None):
    """Per-Gaussian float64 quantities for the renderer, restricted to the
    Gaussians that pass the paper's culling (and the crop cull if asked).
    ``filter_var``: the 3D filter's per-Gaussian variance (or None);
    ``settings.baked``: the inputs hold activated values."""
    means = _f64(means)
    pre = splat.prepare(means, log_scales, quats, opacity_logits, cam, settings.tau_alpha,
                        filter_var, getattr(settings, 'baked', False))
    keep = pre['visible']
    if cull:
        keep = keep & frustum_candidates(pre, cam)
    idx = torch.nonzero(keep).flatten()
    center = torch.as_tensor(cam.center, dtype=F64)
    col = sh.colour(_f64(sh_coeffs)[idx], means[idx], center, sh_degree)
    return Prepared(idx, pre['o'][idx], pre['rho_c'][idx], pre['Tp'][idx], pre['MT'][idx], col)


def evaluate(prep: Prepared, xs, ys, settings):
    """Steps 3-4 for window coordinates xs, ys [P]: returns rho^2, depth,
    fragment mask, alpha before and after the clamp, all [P,G]."""
    pi_x, pi_y = rays.pixel_planes(xs, ys)
    a = rays.to_splat_space(prep.Tp, pi_x)
    b = rays.to_splat_space(prep.Tp, pi_y)
    d, m = rays.pluecker(a, b)
    rho2, z, hit = rays.rho2_and_depth(d, m, prep.MT)
    frag = hit & (rho2 <= prep.rho_c[None, :])
    rho2_safe = torch.where(frag, rho2, torch.zeros_like(rho2))
    raw = prep.o[None, :] * torch.exp(-0.5 * rho2_safe)
    alpha = torch.where(frag, torch.clamp(raw, max=settings.alpha_max), torch.zeros_like(raw))
    return rho2, z, frag, raw, alpha


def render(means, log_scales, quats, opacity_logits, sh_coeffs, sh_degree, cam, settings,
           cull=True, chunk=256, info=False, near_band=1e-3, filter_var=None):
    """Render ``cam`` (whole window). Returns the image [3,H,W] (float64,
    differentiable w.r.t. any parameter tensor passed with requires_grad)
    and, if ``info``, per-pixel fragment records for parity checks. The
    info's ``core`` is [H,W,K] core Gaussian ids for hybrid transparency;
    with sorted blending it is [H,W,2]: the number of blended fragments
    and the id of the fragment the early stop left out (-1 if none)."""
    prep = prepare(means, log_scales, quats, opacity_logits, sh_coeffs, sh_degree, cam,
                   settings, cull, filter_var)
    W, H = int(cam.width), int(cam.height)
    jj, ii = torch.meshgrid(torch.arange(H, dtype=F64), torch.arange(W, dtype=F64),
                            indexing='ij')
    xs_all = (ii + 0.5).flatten()
    ys_all = (jj + 0.5).flatten()
    G = int(prep.idx.numel())
    sorted_mode = bool(getattr(settings, 'sorted_blend', False))
    if sorted_mode:
        # the Gaussians front to back by the view depth of their means
        # (float32, as a per-Gaussian sort key), ties by index
        order = blend.depth_order(splat.mean_view_depth32(means, cam)[prep.idx.numpy()])
    outs, core_list, recs = [], [], []
    for start in range(0, H * W, chunk):
        xs = xs_all[start:start + chunk]
        ys = ys_all[start:start + chunk]
        if G == 0:
            C = torch.as_tensor(settings.bg, dtype=F64)[None, :].expand(xs.numel(), 3)
            outs.append(C)
            if info:
                core_list.append(torch.full((xs.numel(), max(int(settings.K), 0)), -1))
                recs.append(None)
            continue
        rho2, z, frag, raw, alpha = evaluate(prep, xs, ys, settings)
        if sorted_mode:
            C, nb, stop = blend.sorted_alpha(alpha, prep.colour, frag, order, settings.tau_T,
                                             settings.bg)
            core = torch.stack([nb, stop], 1)
        else:
            C, core = blend.hybrid(alpha, prep.colour, z, frag, settings.K, settings.tau_core,
                                   settings.bg, tail=not getattr(settings, 'no_tail', False))
        outs.append(C)
        if info and sorted_mode:
            gid = prep.idx[stop.clamp(min=0)]
            core_list.append(torch.stack([nb, torch.where(stop >= 0, gid,
                                                          torch.full_like(gid, -1))], 1))
        elif info:
            gid = prep.idx[core.clamp(min=0)]
            core_list.append(torch.where(core >= 0, gid, torch.full_like(gid, -1)))
        if info:
            band = (rho2 <= prep.rho_c[None, :] * (1.0 + near_band)) & torch.isfinite(rho2)
            p_i, g_i = torch.nonzero(band, as_tuple=True)
            recs.append(dict(pix=(p_i + start).numpy(), gid=prep.idx[g_i].numpy(),
                             rho2=rho2.detach()[p_i, g_i].numpy(),
                             rho_c=prep.rho_c.detach()[g_i].numpy(),
                             raw=raw.detach()[p_i, g_i].numpy(),
                             depth=z.detach()[p_i, g_i].numpy(),
                             colour=prep.colour.detach()[g_i].numpy(),
                             frag=frag[p_i, g_i].numpy()))
    img = torch.cat(outs, dim=0).reshape(H, W, 3).permute(2, 0, 1)
    if not info:
        return img
    K = 2 if sorted_mode else max(int(settings.K), 0)
    cores = torch.cat(core_list, dim=0).reshape(H, W, -1)[..., :K] if core_list else None
    frags = _merge_records(recs, H * W)
    return img, dict(core=cores, frags=frags, n_candidates=G)


def _merge_records(recs, n_pix):
    keys = ('pix', 'gid', 'rho2', 'rho_c', 'raw', 'depth', 'colour', 'frag')
    parts = [r for r in recs if r is not None]
    if not parts:
        return {k: np.zeros(0) for k in keys} | {'ptr': np.zeros(n_pix + 1, np.int64)}
    out = {k: np.concatenate([r[k] for r in parts]) for k in keys}
    order = np.lexsort((out['gid'], out['pix']))
    out = {k: v[order] for k, v in out.items()}
    out['ptr'] = np.searchsorted(out['pix'], np.arange(n_pix + 1))
    return out


def render_scene(scene, cam, settings, **kw):
    """Convenience wrapper taking a ``scenes.Scene``-like object."""
    kw.setdefault('filter_var', getattr(scene, 'filter_var', None))
    return render(scene.means, scene.log_scales, scene.quats, scene.opacity_logits,
                  scene.sh, scene.sh_degree, cam, settings, **kw)

