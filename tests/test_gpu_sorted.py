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
from tests import crops, parity

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


def test_sorted_rejects_batches():
    sc, cams, st = scenes.workload_small()
    st = sorted_st(st)
    params = to_dev(sc)
    with pytest.raises(htgs.HTGSError):
        htgs.forward(params, sc.sh_degree, [cams[0], cams[0]], st)


# ---------------------------------------------------------------------------
# Backward of sorted blending
# ---------------------------------------------------------------------------

NAMES = ("means", "log_scales", "quats", "opacity_logits", "sh")


def _sorted_grads(sub, cam, st, target):
    """GPU gradient (through the autograd binding) and the oracle's float64
    autograd gradient of sum(G C) with G = sign(C_oracle - target) / (3 H W),
    near-tie pixels left out on both sides."""
    F64 = torch.float64
    ps = [torch.tensor(a, dtype=F64, requires_grad=True) for a in sub.arrays()]
    ref, info = oracle.render.render(*ps, sub.sh_degree, cam, st, cull=False, info=True)
    refn = ref.detach().numpy()
    G = np.sign(refn - target) / (3 * cam.width * cam.height)
    amb = parity.sorted_ambiguous_pixels(info, cam.height, cam.width, st, order_key(sub, cam))
    G[:, amb] = 0.0
    (ref * torch.tensor(G, dtype=F64)).sum().backward()
    want = [p.grad.numpy() for p in ps]
    params = [torch.tensor(a, device="cuda", requires_grad=True) for a in sub.arrays()]
    img = htgs.render(*params, sub.sh_degree, cam, st)
    (img * torch.tensor(G, dtype=torch.float32, device="cuda")).sum().backward()
    got = [p.grad.cpu().numpy() for p in params]
    return img.detach().cpu().numpy(), refn, got, want, int(amb.sum())


def _check(got, want):
    for name, a, b in zip(NAMES, got, want):
        den = np.linalg.norm(b)
        rel = np.linalg.norm(a - b) / max(den, 1e-30)
        elem = np.abs(a - b).max() / max(np.abs(b).max(), 1e-30)
        log(f"  {name}: |g| {den:.3e}, rel {rel:.2e}, elem {elem:.2e}")
        assert rel <= 1e-3 and elem <= 1e-3, name


@pytest.mark.parametrize("seed,tile,tau_T", [
    (7, (8, 8), 1e-4), (11, (16, 16), 1e-4), (13, (8, 8), 0.2), (17, (16, 8), 0.05),
    (19, (32, 8), 1e-4),
])
def test_sorted_gradients_match_oracle_on_subcrop(seed, tile, tau_T):
    """256 Gaussians of the 720p scene on a 32x32 window (tau_T = 0.2 stops
    most pixels early: the gradient must stop where the image did)."""
    sub, cam, st, target = crops.subcrop_720p(seed)
    st = sorted_st(st, tile_w=tile[0], tile_h=tile[1], tau_T=tau_T, bg=(0.1, 0.2, 0.3))
    log(f"sorted gradients: seed {seed}, tile {tile}, tau_T {tau_T}")
    img, ref, got, want, n_amb = _sorted_grads(sub, cam, st, target)
    log(f"  image max-abs {np.abs(img - ref).max():.2e}, near-tie pixels left out {n_amb}")
    _check(got, want)


def test_sorted_gradients_dense_tiles():
    """Many 64-instance chunks per tile (2,400 Gaussians on 16x16 pixels):
    each pixel's transmittance and colour carries cross the chunks of its
    tile in list order."""
    sub, cam, st, target = crops.subcrop_720p(23, n_sel=300, size=16)
    sub = sub.subset(np.tile(np.arange(300), 8))
    r = np.repeat(np.arange(8), 300)[:, None].astype(np.float32)
    sub.means = (sub.means + r * np.array([0.003, -0.002, 0.004], np.float32)).astype(np.float32)
    sub.opacity_logits = (sub.opacity_logits - 3.0).astype(np.float32)   # deep blending
    for tile in ((8, 8), (16, 8)):
        st2 = sorted_st(st, tile_w=tile[0], tile_h=tile[1], tau_T=1e-4)
        params = to_dev(sub)
        frame = gpu_forward(params, sub, [cam], st2)
        keys, _, _, _ = htgs.export_bins(params, sub.sh_degree, [cam], st2, frame.ws)
        per_tile = np.bincount(np.asarray(keys, dtype=np.int64))
        nb = htgs.state_planes(frame)['n_blended']
        log(f"sorted dense: tile {tile}, instances per tile {per_tile.min()}-{per_tile.max()}, "
            f"blended per pixel up to {int(nb.max())}")
        assert per_tile.min() > 300
        img, ref, got, want, n_amb = _sorted_grads(sub, cam, st2, target)
        log(f"  image max-abs {np.abs(img - ref).max():.2e}, near-tie pixels left out {n_amb}")
        _check(got, want)


def test_sorted_backward_counts_the_blended_fragments_and_is_deterministic():
    sc, cams, st = scenes.workload_1080p()
    st = sorted_st(st, tile_w=8, tile_h=8, cost_order=True, tile_cull=True)
    params = to_dev(sc)
    frame = gpu_forward(params, sc, cams, st)
    G = torch.full_like(frame.images[0], 1e-6)
    g1 = htgs.backward(params, frame, [G])
    fwd, bwd = htgs.fragment_counts(frame.ws)
    nb = int(htgs.state_planes(frame)['n_blended'].sum())
    log(f"sorted 1080p: blended {nb}, forward counter {fwd}, backward {bwd}")
    assert fwd == nb and bwd == nb
    g2 = htgs.backward(params, frame, [G])
    for a, b in zip(g1, g2):
        assert torch.equal(a, b)
        assert torch.isfinite(a).all()
