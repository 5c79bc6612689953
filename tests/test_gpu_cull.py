"""Tile culling on rects with many tile rows (needs an MI355X).

The preprocess tests the tile rows of every small rect (at most 64 tiles) of
a wave together, dealing the (Gaussian, row) pairs to the lanes in windows of
64. The scene here mixes, in random order:
* vertical needles one or two tiles wide and up to ~60 tiles tall (one lane
  with dozens of rows: many windows, owners that span windows);
* thin needles at random angles (diagonal rects that are mostly empty, so
  most of their tiles are culled);
* small round splats (one or two rows);
* Gaussians behind the camera (lanes with nothing to test).

Culling drops only tiles the splat's ellipse never reaches, so the image and
the forward state must equal those of the same frame without culling bit for
bit, with fewer instances; the gradients regroup their per-Gaussian sums and
agree to rounding."""
import dataclasses
import math

import numpy as np
import pytest
import torch

import oracle
from paper_2410_08129_amd import htgs, scenes

pytestmark = pytest.mark.gpu


def log(msg):
    print(msg, flush=True)


W, H = 256, 640
CAM = scenes.look_at((0, 0, -5), (0, 0, 0), (0, -1, 0), 40.0, W, H)


def _needle_scene(seed=0, n=4000):
    rng = np.random.default_rng(seed)
    kind = rng.integers(0, 4, n)       # 0 vertical, 1 angled, 2 round, 3 behind the camera
    depth = rng.uniform(4.0, 6.0, n)   # distance from the eye along the view axis
    px = rng.uniform(0.0, W, n)
    py = rng.uniform(60.0, H - 60.0, n)
    z = depth - 5.0
    z[kind == 3] = -8.0                # behind the eye at z = -5
    x = (px - CAM.cx) / CAM.fx * depth
    y = (py - CAM.cy) / CAM.fy * depth
    means = np.stack([x, y, z], axis=1)
    pix = depth / CAM.fx               # world length of one pixel at the Gaussian's depth
    long_px = np.where(kind == 0, rng.uniform(10.0, 75.0, n),
                       np.where(kind == 1, rng.uniform(4.0, 14.0, n), rng.uniform(1.0, 3.0, n)))
    short_px = np.where(kind == 2, long_px, 0.3)
    ls = np.log(np.stack([long_px * pix, short_px * pix, short_px * pix], axis=1))
    theta = np.where(kind == 0, 0.5 * math.pi, rng.uniform(0.0, math.pi, n))
    # rotation about the view axis by theta takes the long (x) axis to image direction theta
    q = np.stack([np.cos(theta / 2), np.zeros(n), np.zeros(n), np.sin(theta / 2)], axis=1)
    logit = rng.normal(1.0, 0.5, n)
    sh = np.zeros((n, 1, 3))
    sh[:, 0, :] = rng.uniform(-1.0, 1.0, (n, 3))
    return scenes._pack(means, ls, q, logit, sh, 0)


def _render(params, sc, st, G):
    frame = htgs.forward(params, sc.sh_degree, [CAM], st)
    grads = htgs.backward(params, frame, [G])
    torch.cuda.synchronize()
    flags, n_inst = htgs.read_status(frame.ws)
    assert flags == 0, flags
    return frame, grads, htgs.state_planes(frame, 0), n_inst


@pytest.mark.parametrize("seed", [0, 1])
def test_cull_with_tall_rects_keeps_every_fragment(seed):
    sc = _needle_scene(seed)
    st = scenes.RenderSettings(K=4, tile_w=8, tile_h=8)
    # the rects the cull sees: tile rows of those with 2..64 tiles
    prep = oracle.splat.prepare(sc.means, sc.log_scales, sc.quats, sc.opacity_logits, CAM,
                                st.tau_alpha, None, False)
    rect, ok, _ = oracle.bins.pixel_rects(prep, CAM)
    rows = rect[ok, 3] // 8 - rect[ok, 1] // 8 + 1
    cnt = (rect[ok, 2] // 8 - rect[ok, 0] // 8 + 1) * rows
    tested = rows[(cnt >= 2) & (cnt <= 64)]
    log(f"seed {seed}: {int(ok.sum())} of {sc.n} visible, {tested.size} rects culled, "
        f"rows mean {tested.mean():.2f} max {int(tested.max())}")
    assert tested.max() >= 40

    params = [torch.tensor(a, device="cuda") for a in sc.arrays()]
    G = torch.tensor(np.random.default_rng(seed + 5).normal(0, 1, (3, H, W)),
                     dtype=torch.float32, device="cuda")
    f0, g0, p0, n0 = _render(params, sc, st, G)
    f1, g1, p1, n1 = _render(params, sc, dataclasses.replace(st, tile_cull=True), G)
    log(f"  instances {n0} without culling, {n1} with")
    assert n1 < n0
    assert torch.equal(f0.images[0], f1.images[0])
    for k in ("core_ids", "core_alpha", "T", "A", "S", "P"):
        assert torch.equal(p0[k], p1[k]), k
    for a, b in zip(g0, g1):
        assert float((a - b).norm()) <= 1e-5 * max(float(b.norm()), 1e-30)
