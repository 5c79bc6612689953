"""Sorted blending (the paper's "w/o per-pixel HT" configuration, Sec. 4.3,
Table splat_eval) on the HIP path against the float64 oracle, through the C
ABI (needs an MI355X).

Bar: depth-ordered tile lists bit-exact (the front-to-back order of the
means' float32 view depths inside every tile, ties by index); images within
1e-4 max-abs, with each pixel's blended-fragment count and stop Gaussian
equal to the oracle's except at near-ties (tests/parity.py decides those by
recomputing the GPU's branch in float64)."""
import dataclasses

import numpy as np
import pytest
import torch

import oracle
from paper_2410_08129_amd import htgs, scenes
from tests import parity

pytestmark = pytest.mark.gpu


def log(msg):
    print(msg, flush=True)


def to_dev(sc):
    return [torch.tensor(a, device="cuda") for a in sc.arrays()]


def sorted_st(st, **kw):
    return dataclasses.replace(st, sorted_blend=True, **kw)


def gpu_forward(params, sc, cams, st, with_state=True):
    frame = htgs.forward(params, sc.sh_degree, cams, st, with_state=with_state)
    torch.cuda.synchronize()
    flags, n = htgs.read_status(frame.ws)
    assert flags == 0, flags
    return frame


def order_key(sc, cam):
    return oracle.splat.mean_view_depth32(sc.means, cam)


def check_window(sc, cam_full, frame, st, x0, y0, w, h):
    """The GPU frame's window [x0, x0+w) x [y0, y0+h) against the oracle."""
    planes = htgs.state_planes(frame)
    img = frame.images[0].cpu().numpy()[:, y0:y0 + h, x0:x0 + w]
    nb = planes['n_blended'].cpu().numpy()[y0:y0 + h, x0:x0 + w]
    stop = planes['stop_id'].cpu().numpy()[y0:y0 + h, x0:x0 + w]
    cam = cam_full.crop(x0, y0, w, h)
    ref, info = oracle.render.render_scene(sc, cam, st, info=True)
    return parity.check_sorted_image(img, nb, stop, ref.numpy(), info, order_key(sc, cam_full), st)


@pytest.mark.parametrize("tile", [(16, 16), (8, 8), (16, 8), (32, 8)])
def test_small_sorted_tile_lists_bit_exact(tile):
    sc, cams, st = scenes.workload_small()
    st = sorted_st(st, tile_w=tile[0], tile_h=tile[1])
    log(f"sorted bins, small scene, tile {tile}")
    params = to_dev(sc)
    frame = gpu_forward(params, sc, cams, st)
    keys, vals, rects, _ = htgs.export_bins(params, sc.sh_degree, cams, st, frame.ws)
    ref = oracle.bins.tile_lists(sc.means, sc.log_scales, sc.quats, sc.opacity_logits, cams[0], st)
    n_amb = parity.compare_bins(keys, vals, rects, ref)
    log(f"  instances {len(keys)}, round-off ties {n_amb}")


def test_1080p_sorted_tile_lists_bit_exact():
    """1M Gaussians: the depth sort of all means and the stable tile sort of
    the depth-ordered instances give exactly the oracle's lists."""
    sc, cams, st = scenes.workload_1080p()
    st = sorted_st(st, tile_w=8, tile_h=8)
    log("sorted bins, 1080p, 8x8")
    params = to_dev(sc)
    frame = gpu_forward(params, sc, cams, st, with_state=False)
    keys, vals, rects, _ = htgs.export_bins(params, sc.sh_degree, cams, st, frame.ws)
    ref = oracle.bins.tile_lists(sc.means, sc.log_scales, sc.quats, sc.opacity_logits, cams[0], st)
    n_amb = parity.compare_bins(keys, vals, rects, ref)
    log(f"  instances {len(keys)}, round-off ties {n_amb}")


@pytest.mark.parametrize("tile,tau_T,bg", [
    ((16, 16), 1e-4, (0.0, 0.0, 0.0)), ((8, 8), 1e-4, (0.2, 0.4, 0.6)),
    ((8, 8), 0.3, (0.1, 0.1, 0.1)), ((16, 8), 0.05, (0.0, 0.5, 0.0)),
    ((32, 8), 1e-4, (0.3, 0.0, 0.2)), ((8, 8), 0.0, (0.0, 0.0, 0.0)),
])
def test_small_sorted_image_parity(tile, tau_T, bg):
    """Full 128x128 frame and a ragged crop, several stop thresholds (0.3
    stops most pixels after a few fragments; 0 never stops)."""
    sc, cams, st = scenes.workload_small()
    st = sorted_st(st, tile_w=tile[0], tile_h=tile[1], tau_T=tau_T, bg=bg, cost_order=True)
    params = to_dev(sc)
    for cam, label in ((cams[0], "full"), (cams[0].crop(21, 37, 77, 53), "crop")):
        log(f"sorted image, small {label}, tile {tile}, tau_T {tau_T}")
        frame = gpu_forward(params, sc, [cam], st)
        stats = check_window(sc, cam, frame, st, 0, 0, cam.width, cam.height)
        nb = htgs.state_planes(frame)['n_blended']
        fwd, _ = htgs.fragment_counts(frame.ws)
        log(f"  {stats}; blended fragments {int(nb.sum())} (counter {fwd})")
        assert stats['max_err_clean'] < 1e-4
        assert int(nb.sum()) == fwd


def test_small_sorted_early_stop_changes_the_image():
    sc, cams, st = scenes.workload_small()
    params = to_dev(sc)
    a = gpu_forward(params, sc, cams, sorted_st(st, tau_T=0.0)).images[0]
    b = gpu_forward(params, sc, cams, sorted_st(st, tau_T=0.5)).images[0]
    assert float((a - b).abs().max()) > 1e-2


def test_1080p_sorted_image_crops():
    sc, cams, st = scenes.workload_1080p()
    st = sorted_st(st, tile_w=8, tile_h=8, cost_order=True, tile_cull=True)
    log("sorted 1080p full frame, 3 crops of 64x64 vs oracle")
    params = to_dev(sc)
    frame = gpu_forward(params, sc, cams, st)
    crops = [(928, 508)] + [(x, y) for x, y, _ in scenes.random_crops(cams[0], 2, 64, seed=3)]
    for (x0, y0) in crops:
        stats = check_window(sc, cams[0], frame, st, x0, y0, 64, 64)
        log(f"  crop ({x0},{y0}): {stats}")
        assert stats['max_err_clean'] < 1e-4


def test_sorted_persistent_and_cull_schedules_match():
    """The persistent tile queue and tile culling leave the sorted image,
    counts and stops bit-identical (culled tiles hold no fragment)."""
    sc, cams, st = scenes.workload_small()
    st = sorted_st(st, tile_w=8, tile_h=8)
    params = to_dev(sc)
    base = gpu_forward(params, sc, cams, st)
    for kw in (dict(persistent=True), dict(tile_cull=True), dict(cost_order=True, persistent=True)):
        other = gpu_forward(params, sc, cams, dataclasses.replace(st, **kw))
        assert torch.equal(base.images[0], other.images[0]), kw
        pa, pb = htgs.state_planes(base), htgs.state_planes(other)
        for k in ("n_blended", "stop_id", "end_pos"):
            if k == "end_pos" and kw.get("tile_cull"):
                continue   # list positions move when tiles drop instances
            assert torch.equal(pa[k], pb[k]), (kw, k)


def test_sorted_rejects_backward_and_batches():
    sc, cams, st = scenes.workload_small()
    st = sorted_st(st)
    params = to_dev(sc)
    frame = gpu_forward(params, sc, cams, st)
    with pytest.raises(htgs.HTGSError):
        htgs.backward(params, frame, [torch.ones_like(frame.images[0])])
    with pytest.raises(htgs.HTGSError):
        htgs.forward(params, sc.sh_degree, [cams[0], cams[0]], st)
