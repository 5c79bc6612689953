"""The batched multi-view path against the FP64 oracle, through the C ABI
(needs an MI355X): several views of uneven size, one of them off-axis, in
one htgs_render_forward_batched / htgs_render_backward_batched call.

* each view's image against oracle.render of that view (1e-4 max-abs,
  near-ties through the admissibility protocol);
* the batched tile lists bit-exact against the oracle's per-view lists,
  each view's keys offset by the tile count of the views before it (16-bit
  keys on the small scene; 32-bit keys and three sort passes on four 1080p
  views at 8x8 tiles);
* the batched gradient against the sum over the views of the oracle's
  float64 autograd gradients (1e-3 relative, norm and element-wise)."""
import dataclasses

import numpy as np
import pytest
import torch

import oracle
from paper_2410_08129_amd import htgs, scenes
from tests import crops, parity

pytestmark = pytest.mark.gpu

F64 = torch.float64
NAMES = ("means", "log_scales", "quats", "opacity_logits", "sh")


def log(msg):
    print(msg, flush=True)


def to_dev(sc):
    return [torch.tensor(a, device="cuda") for a in sc.arrays()]


def small_views():
    sc, cams, st = scenes.workload_small()
    views = [cams[0].crop(9, 23, 101, 77),                                        # off-axis
             scenes.look_at((1.5, -1.0, -2.5), (0, 0, 0), (0, -1, 0), 50.0, 90, 70),
             scenes.look_at((-2.0, 0.5, -2.2), (0.1, 0, 0), (0, -1, 0), 65.0, 128, 96)]
    return sc, views


def oracle_batched_lists(sc, views, st):
    keys, vals, amb = [], [], []
    base = 0
    for v in views:
        ref = oracle.bins.tile_lists(sc.means, sc.log_scales, sc.quats, sc.opacity_logits, v, st)
        keys.append(ref['keys'] + base)
        vals.append(ref['values'])
        amb.append(np.nonzero(ref['margin'] < 1e-9)[0])
        base += ref['tiles_x'] * ref['tiles_y']
    return np.concatenate(keys), np.concatenate(vals), np.unique(np.concatenate(amb)), base


def compare_batched_lists(gk, gv, rk, rv, amb):
    gk, gv = gk.astype(np.int64), gv.astype(np.int64)
    if amb.size:
        kg, kr = ~np.isin(gv, amb), ~np.isin(rv, amb)
        gk, gv, rk, rv = gk[kg], gv[kg], rk[kr], rv[kr]
    assert gk.shape == rk.shape, (gk.shape, rk.shape)
    assert (gk == rk).all() and (gv == rv).all(), "batched lists differ"


@pytest.mark.parametrize("K,tile,cull", [(4, 16, False), (8, 8, True)])
def test_batched_images_match_oracle(K, tile, cull):
    sc, views = small_views()
    st = scenes.RenderSettings(K=K, tile_w=tile, tile_h=tile, tile_cull=cull, cost_order=cull,
                               bg=(0.05, 0.1, 0.2))
    log(f"batched images: 3 views {[(v.width, v.height) for v in views]}, K={K}, tile={tile}")
    params = to_dev(sc)
    frame = htgs.forward(params, sc.sh_degree, views, st)
    torch.cuda.synchronize()
    assert htgs.read_status(frame.ws)[0] == 0
    for i, v in enumerate(views):
        ref, info = oracle.render.render_scene(sc, v, st, info=True)
        stats = parity.check_image(frame.images[i].cpu().numpy(),
                                   htgs.state_planes(frame, i)['core_ids'].cpu().numpy(),
                                   ref.numpy(), info, st)
        log(f"  view {i}: {stats}")
        assert stats['max_err_clean'] < 1e-4


def test_batched_lists_bit_exact_16bit():
    sc, views = small_views()
    st = scenes.RenderSettings(K=4, tile_w=16, tile_h=16)
    params = to_dev(sc)
    frame = htgs.forward(params, sc.sh_degree, views, st, with_state=False)
    keys, vals, _, _ = htgs.export_bins(params, sc.sh_degree, views, st, frame.ws)
    rk, rv, amb, tiles = oracle_batched_lists(sc, views, st)
    assert tiles <= 65536
    compare_batched_lists(keys, vals, rk, rv, amb)
    log(f"  batched 16-bit lists: {len(keys)} instances, {tiles} tiles, ties {amb.size}")


def test_batched_lists_bit_exact_32bit_keys():
    sc = scenes.clustered_scene(200_000, 64, seed=4)
    views = [scenes.look_at(e, (0, 0, 0), (0, -1, 0), 50.0, 1920, 1080)
             for e in ((0, 0, -25), (6, -3, -23), (-20, 2, -14), (12, 10, 19))]
    st = scenes.RenderSettings(K=8, tile_w=8, tile_h=8)
    params = to_dev(sc)
    log("batched lists: 200k Gaussians, 4 views of 1920x1080, 8x8 tiles")
    frame = htgs.forward(params, sc.sh_degree, views, st, with_state=False)
    keys, vals, _, flags = htgs.export_bins(params, sc.sh_degree, views, st, frame.ws)
    assert flags == 0
    rk, rv, amb, tiles = oracle_batched_lists(sc, views, st)
    assert tiles > 65536       # 17-bit keys: 32-bit key arrays, three sort passes
    compare_batched_lists(keys, vals, rk, rv, amb)
    log(f"  batched 32-bit lists: {len(keys)} instances, {tiles} tiles, ties {amb.size}")


def gradient_views(seed):
    """256 Gaussians of a 720p window and three small views of them: the
    720p camera's own 32x32 window (off-axis: its principal point lies
    outside the image) and two cameras a few degrees to either side,
    looking at the sample's centre, of uneven sizes."""
    sub, cam, st, _ = crops.subcrop_720p(seed)
    centre = sub.means.astype(np.float64).mean(0)
    eye0 = cam.center
    d = centre - eye0
    dist = np.linalg.norm(d)
    side = np.cross(d / dist, (0.0, -1.0, 0.0))
    side /= np.linalg.norm(side)
    views = [cam]
    for ang, (w, h) in ((0.05, (40, 28)), (-0.07, (27, 45))):
        eye = centre - np.cos(ang) * d + np.sin(ang) * dist * side
        views.append(scenes.look_at(eye, centre, (0, -1, 0), 2.2, w, h))
    return sub, views, st


@pytest.mark.parametrize("seed,tile", [(7, 8), (13, 16)])
def test_batched_gradient_is_the_sum_of_oracle_view_gradients(seed, tile):
    sub, views, st = gradient_views(seed)
    st = dataclasses.replace(st, tile_w=tile, tile_h=tile, cost_order=True, tile_cull=True)
    rng = np.random.default_rng(seed)
    Gs = [rng.normal(0, 1, (3, v.height, v.width)) / (3 * v.width * v.height) for v in views]
    # oracle: one float64 autograd pass per view, summed
    ref = [np.zeros(a.shape) for a in sub.arrays()]
    ps = [torch.tensor(a, dtype=F64, requires_grad=True) for a in sub.arrays()]
    masks = []
    for v, G in zip(views, Gs):
        img, info = oracle.render.render(*[torch.tensor(a) for a in sub.arrays()], sub.sh_degree,
                                         v, st, cull=False, info=True)
        amb = parity.ambiguous_pixels(info, v.height, v.width, st)
        masks.append(amb)
        G[:, amb] = 0.0
        img = oracle.render.render(*ps, sub.sh_degree, v, st, cull=False)
        (img * torch.tensor(G, dtype=F64)).sum().backward()
    ref = [p.grad.numpy() for p in ps]
    log(f"batched gradients: seed {seed}, tile {tile}, views {[(v.width, v.height) for v in views]}"
        f", near-tie pixels left out {[int(m.sum()) for m in masks]}")
    params = to_dev(sub)
    frame = htgs.forward(params, sub.sh_degree, views, st)
    grads = htgs.backward(params, frame, [torch.tensor(G, dtype=torch.float32, device="cuda")
                                          for G in Gs])
    torch.cuda.synchronize()
    assert htgs.read_status(frame.ws)[0] == 0
    for name, (den, rel, elem) in zip(NAMES, parity.grad_errors(
            [g.cpu().numpy() for g in grads], ref)):
        log(f"  {name}: |g| {den:.3e}, rel {rel:.2e}, elem {elem:.2e}")
        assert rel <= 1e-3 and elem <= 1e-3, name
