"""Tile/key-list reference (paper Sec. 4.3, "tiling": per-tile primitive lists
keyed by a tile id, with no depth sort).

For every Gaussian that survives culling, the float64 screen box
[p - h, p + h] of Sec. 3.2 is turned into the range of pixels whose centres
lie inside it, i in [ceil(b_x - 1/2), floor(t_x - 1/2)] clamped to
[0, W - 1] (same for rows), and then into the range of tiles those pixels
fall in. Each (Gaussian, tile) pair is one instance with key = row-major tile
id and value = Gaussian index; the list is ordered by key and, within a key,
by ascending Gaussian index. The margin of a Gaussian is the smallest
distance of its four box edges (minus 1/2) from an integer; a disagreement
about a rect with a margin above 1e-9 is a real bug, below it a round-off tie.

For sorted blending (the paper's "w/o per-pixel HT" configuration, Sec. 4.3
and Table splat_eval) each tile's list is instead ordered front to back by
the view depth of the Gaussians' means, as a float32 key (3DGS's order),
ties by ascending index.
"""
from __future__ import annotations

import math

import numpy as np

from . import splat


def pixel_rects(prep, cam):
    """Inclusive pixel ranges [x0, y0, x1, y1] per Gaussian (int64), a mask
    of non-empty ranges, and the per-Gaussian edge margin."""
    p = prep['p'].detach().numpy()
    h = prep['h'].detach().numpy()
    vis = prep['visible'].numpy()
    n = p.shape[0]
    rect = np.zeros((n, 4), np.int64)
    margin = np.full(n, np.inf)
    ok = np.zeros(n, bool)
    idx = np.nonzero(vis)[0]
    lo = p[idx, :2] - h[idx, :2] - 0.5
    hi = p[idx, :2] + h[idx, :2] - 0.5
    x0 = np.maximum(np.ceil(lo[:, 0]), 0.0)
    y0 = np.maximum(np.ceil(lo[:, 1]), 0.0)
    x1 = np.minimum(np.floor(hi[:, 0]), cam.width - 1.0)
    y1 = np.minimum(np.floor(hi[:, 1]), cam.height - 1.0)
    good = (x0 <= x1) & (y0 <= y1)
    sel = idx[good]
    ok[sel] = True
    rect[sel] = np.stack([x0, y0, x1, y1], 1)[good].astype(np.int64)
    edges = np.concatenate([lo, hi], 1)
    margin[idx] = np.abs(edges - np.round(edges)).min(1)
    return rect, ok, margin


def tile_lists(means, log_scales, quats, opacity_logits, cam, settings, filter_var=None):
    """Sorted (keys, values) of all instances, the per-Gaussian tile rects
    [tx0, ty0, tx1, ty1] (inclusive, -1 where empty) and edge margins."""
    prep = splat.prepare(means, log_scales, quats, opacity_logits, cam, settings.tau_alpha,
                         filter_var, getattr(settings, 'baked', False))
    rect, ok, margin = pixel_rects(prep, cam)
    tw, th = int(settings.tile_w), int(settings.tile_h)
    tiles_x = math.ceil(cam.width / tw)
    trect = np.full((rect.shape[0], 4), -1, np.int64)
    trect[ok, 0] = rect[ok, 0] // tw
    trect[ok, 1] = rect[ok, 1] // th
    trect[ok, 2] = rect[ok, 2] // tw
    trect[ok, 3] = rect[ok, 3] // th
    g = np.nonzero(ok)[0]
    w = trect[g, 2] - trect[g, 0] + 1
    cnt = w * (trect[g, 3] - trect[g, 1] + 1)
    owner = np.repeat(g, cnt)
    start = np.repeat(np.cumsum(cnt) - cnt, cnt)
    rank = np.arange(owner.size) - start
    wr = np.repeat(w, cnt)
    tx = trect[owner, 0] + rank % wr
    ty = trect[owner, 1] + rank // wr
    keys = ty * tiles_x + tx
    zkey = None
    if getattr(settings, 'sorted_blend', False):
        # sorted blending: inside a tile, front to back by the float32 view
        # depth of the means, ties by index (3DGS's per-tile order)
        zkey = splat.mean_view_depth32(means, cam)
        order = np.lexsort((owner, zkey[owner], keys))
    else:
        order = np.lexsort((owner, keys))
    counts = np.zeros(rect.shape[0], np.int64)
    counts[g] = cnt
    return dict(keys=keys[order], values=owner[order], tile_rect=trect, pixel_rect=rect,
                nonempty=ok, margin=margin, counts=counts, tiles_x=tiles_x,
                tiles_y=math.ceil(cam.height / th), depth32=zkey)

