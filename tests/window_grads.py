"""Gradient windows at full scene density (test code, float64 oracle).

The GPU renders the whole frame with every Gaussian of the scene, under a
given schedule, and back-propagates a loss whose weights are zero outside
a few windows; the oracle renders only the Gaussians whose float64 screen
box meets a window (no other Gaussian reaches its pixels) and
back-propagates the same weights, 16x16 pixels at a time (the loss is a
sum over pixels, so the pieces add up to the window's gradient). Pixels
holding a near-tie are left out of the loss on both sides (their branch
is not decided by float64 alone)."""
from __future__ import annotations

import numpy as np
import torch

import oracle
from tests import crops, parity

F64 = torch.float64


def oracle_window(sc, cam, st, x0, y0, wdt, hgt, G_full, p, h, vis, piece=16):
    """Oracle image and core of one window, its near-tie mask (the window's
    pixels of G_full at near-ties are set to zero in place) and the float64
    gradient of sum(G_full * C) over the window, as (indices, grads)."""
    idx = crops.meeting(p, h, vis, x0, y0, wdt, hgt)
    sub = sc.subset(idx)
    win = cam.crop(x0, y0, wdt, hgt)
    ref, info = oracle.render.render(*[torch.tensor(a) for a in sub.arrays()], sub.sh_degree, win,
                                     st, cull=True, info=True)
    amb = parity.ambiguous_pixels(info, hgt, wdt, st)
    Gw = G_full[:, y0:y0 + hgt, x0:x0 + wdt]
    Gw[:, amb] = 0.0
    ps = [torch.tensor(a, dtype=F64, requires_grad=True) for a in sub.arrays()]
    for sy in range(0, hgt, piece):
        for sx in range(0, wdt, piece):
            g = Gw[:, sy:sy + piece, sx:sx + piece]
            if not np.any(g):
                continue
            im = oracle.render.render(*ps, sub.sh_degree,
                                      cam.crop(x0 + sx, y0 + sy, g.shape[2], g.shape[1]),
                                      st, cull=True)
            (im * torch.tensor(g, dtype=F64)).sum().backward()
    grads = [p_.grad.numpy() if p_.grad is not None else np.zeros(p_.shape) for p_ in ps]
    return dict(idx=idx, ref=ref.numpy(), info=info, amb=amb, grads=grads,
                frags_per_px=float(info['frags']['frag'].sum()) / (wdt * hgt))


def accumulate(n, shapes, windows):
    """Sum of the windows' oracle gradients as full [n, ...] arrays, and the
    mask of Gaussians any window touches."""
    out = [np.zeros((n,) + s) for s in shapes]
    touched = np.zeros(n, bool)
    for w in windows:
        for o, g in zip(out, w['grads']):
            np.add.at(o, w['idx'], g)
        touched[w['idx']] = True
    return out, touched
