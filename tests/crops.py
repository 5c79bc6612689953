"""Seeded gradient windows of the 720p workload (test code).

A window is centred on a seeded random visible Gaussian's projected mean;
its Gaussians are a seeded sample of those whose float64 screen box meets
the window. The box comes from the oracle (its pinned bound), so no
Gaussian outside the sample reaches the window."""
from __future__ import annotations

import numpy as np

import oracle
from paper_2410_08129_amd import scenes

_CACHE = {}


def _scene_720p():
    if '720p' not in _CACHE:
        sc, cams, st = scenes.workload_720p()
        cam = cams[0]
        pre = oracle.splat.prepare(sc.means, sc.log_scales, sc.quats, sc.opacity_logits, cam,
                                   st.tau_alpha)
        _CACHE['720p'] = (sc, cam, st, pre['p'].numpy(), pre['h'].numpy(),
                          pre['visible'].numpy())
    return _CACHE['720p']


def meeting(p, h, vis, x0, y0, w, hgt):
    """Indices of the visible Gaussians whose box [p - h, p + h] meets the
    pixel window [x0, x0 + w) x [y0, y0 + hgt)."""
    return np.nonzero(vis & (p[:, 0] + h[:, 0] >= x0) & (p[:, 0] - h[:, 0] <= x0 + w)
                      & (p[:, 1] + h[:, 1] >= y0) & (p[:, 1] - h[:, 1] <= y0 + hgt))[0]


def subcrop_720p(seed=7, n_sel=256, size=32):
    """(subset scene, crop camera, settings, target window) of the 720p
    workload: n_sel Gaussians on a size x size window."""
    sc, cam, st, p, h, vis = _scene_720p()
    rng = np.random.default_rng(seed)
    inner = np.nonzero(vis & (p[:, 0] > 40) & (p[:, 0] < cam.width - 40) & (p[:, 1] > 40)
                       & (p[:, 1] < cam.height - 40))[0]
    while True:
        g = int(rng.choice(inner))
        x0 = int(round(p[g, 0])) - size // 2
        y0 = int(round(p[g, 1])) - size // 2
        meets = meeting(p, h, vis, x0, y0, size, size)
        if meets.size >= n_sel:
            break
    sel = np.sort(rng.choice(meets, n_sel, replace=False))
    target = scenes.smooth_target(cam.height, cam.width)[:, y0:y0 + size, x0:x0 + size]
    st = scenes.RenderSettings(**{f: getattr(st, f) for f in st.__dataclass_fields__})
    return sc.subset(sel), cam.crop(x0, y0, size, size), st, target
