"""Tile lists on key distributions that stress the binning launches (needs an
MI355X), bit-exact against the FP64 oracle's lists.

* One tile: thousands of tiny splats inside one 8x8 tile, so every key is
  the same (every wave of the digit counts holds a single digit; every
  chunk of the scatter is one digit run).
* Mostly empty: most Gaussians behind the camera or outside the frustum,
  interleaved with a few that cover many tiles (emit windows whose owners
  lie past long runs of empty entries).
* Raster order: splats on a grid, indexed row by row, so that neighbouring
  instances share tile digits (repeated digits inside waves, not all equal).
* Few instances: fewer than one sort chunk of 4,096 keys, and a few
  chunks with a partial last one."""
import numpy as np
import pytest
import torch

import oracle
from paper_2410_08129_amd import htgs, scenes
from tests import parity

pytestmark = pytest.mark.gpu


def log(msg):
    print(msg, flush=True)


CAM = scenes.look_at((0, 0, -5), (0, 0, 0), (0, -1, 0), 60.0, 320, 240)


def _scene(means, log_scale, seed=0):
    rng = np.random.default_rng(seed)
    n = means.shape[0]
    ls = np.broadcast_to(np.asarray(log_scale, np.float64), (n, 3)).copy()
    q = rng.normal(0.0, 1.0, (n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    logit = rng.normal(1.0, 0.5, n)
    sh = np.zeros((n, 1, 3))
    sh[:, 0, :] = rng.uniform(-1.0, 1.0, (n, 3))
    return scenes._pack(means, ls, q, logit, sh, 0)


def _unproject(px, py, depth, cam=CAM):
    """World points at pixel (px, py) and view depth `depth`."""
    x = (np.asarray(px, np.float64) - cam.cx) / cam.fx * depth
    y = (np.asarray(py, np.float64) - cam.cy) / cam.fy * depth
    pc = np.stack([x, y, np.broadcast_to(depth, np.shape(x))], axis=1)
    R = cam.world_to_cam[:, :3].astype(np.float64)
    t = cam.world_to_cam[:, 3].astype(np.float64)
    return (pc - t) @ R    # R^T (pc - t)


def _check(sc, tile=8, **kw):
    st = scenes.RenderSettings(K=4, tile_w=tile, tile_h=tile, **kw)
    params = [torch.tensor(a, device="cuda") for a in sc.arrays()]
    frame = htgs.forward(params, sc.sh_degree, [CAM], st, with_state=False)
    torch.cuda.synchronize()
    flags, n_inst = htgs.read_status(frame.ws)
    assert flags == 0, flags
    keys, vals, rects, _ = htgs.export_bins(params, sc.sh_degree, [CAM], st, frame.ws)
    ref = oracle.bins.tile_lists(sc.means, sc.log_scales, sc.quats, sc.opacity_logits, CAM, st)
    n_amb = parity.compare_bins(keys, vals, rects, ref)
    return keys, n_amb


def test_single_tile_all_keys_equal():
    rng = np.random.default_rng(1)
    n = 20000
    px = rng.uniform(162.5, 165.5, n)   # boxes inside tile column 20 of 8-pixel tiles
    py = rng.uniform(82.5, 85.5, n)     # and tile row 10
    means = _unproject(px, py, rng.uniform(3.0, 6.0, n))
    sc = _scene(means, -5.5)
    keys, n_amb = _check(sc)
    log(f"one tile: {len(keys)} instances, ties {n_amb}")
    assert len(keys) > 4 * 4096     # several full chunks of one key
    assert len(np.unique(keys)) == 1


def test_mostly_empty_entries():
    rng = np.random.default_rng(2)
    n = 60000
    px = rng.uniform(-200.0, 520.0, n)
    py = rng.uniform(-200.0, 440.0, n)
    depth = rng.uniform(2.0, 8.0, n)
    behind = rng.uniform(0.0, 1.0, n) < 0.6
    depth[behind] = -depth[behind]     # behind the camera: no instance
    means = _unproject(px, py, depth)
    ls = np.full(n, -6.0)
    big = rng.choice(n, 400, replace=False)
    ls[big] = -1.0                     # up to hundreds of tiles each
    sc = _scene(means, ls[:, None])
    keys, n_amb = _check(sc)
    n_inst = len(keys)
    per = np.asarray(oracle.bins.tile_lists(sc.means, sc.log_scales, sc.quats, sc.opacity_logits,
                                            CAM, scenes.RenderSettings(K=4, tile_w=8, tile_h=8))
                     ['counts'])
    log(f"mostly empty: {n_inst} instances, {int((per == 0).sum())} of {n} Gaussians without "
        f"one, max {int(per.max())} per Gaussian, ties {n_amb}")
    assert (per == 0).mean() > 0.5 and per.max() > 64


@pytest.mark.parametrize("tile", [8, 16])
def test_raster_order_repeated_digits(tile):
    xs, ys = np.meshgrid(np.linspace(2.0, 317.0, 240), np.linspace(2.0, 237.0, 180))
    means = _unproject(xs.ravel(), ys.ravel(), 4.0)
    sc = _scene(means, -4.5)
    keys, n_amb = _check(sc, tile=tile)
    log(f"raster order, tile {tile}: {len(keys)} instances, ties {n_amb}")
    assert len(keys) > 2 * 4096


@pytest.mark.parametrize("n", [37, 700])
def test_few_instances(n):
    rng = np.random.default_rng(3 + n)
    means = _unproject(rng.uniform(0.0, 320.0, n), rng.uniform(0.0, 240.0, n),
                       rng.uniform(2.0, 8.0, n))
    sc = _scene(means, -3.5)
    keys, n_amb = _check(sc)
    log(f"{n} Gaussians: {len(keys)} instances, ties {n_amb}")
    assert len(keys) > 0


@pytest.mark.parametrize("levels", [1, 3])
def test_sorted_lists_with_depth_ties(levels):
    """Sorted blending's lists when many means share one view depth: the
    depth sort is stable, so ties stay in index order (all depth keys equal
    for one level)."""
    xs, ys = np.meshgrid(np.linspace(2.0, 317.0, 160), np.linspace(2.0, 237.0, 120))
    n = xs.size
    depth = 3.0 + np.arange(n) % levels
    means = _unproject(xs.ravel(), ys.ravel(), depth)
    sc = _scene(means, -4.0)
    keys, n_amb = _check(sc, sorted_blend=True)
    log(f"sorted, {levels} depth level(s): {len(keys)} instances, ties {n_amb}")
    assert len(keys) > 4096
