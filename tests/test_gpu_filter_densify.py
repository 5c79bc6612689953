"""Input and training-side options of the HIP path against the FP64 oracle
(needs an MI355X): the 3D smoothing filter (images and gradients), baked
inputs (images), the densification statistic and view counts of the
backward, and the opacity decay kernel."""
import dataclasses

import numpy as np
import pytest
import torch

import oracle
from paper_2410_08129_amd import htgs, scenes
from tests import crops, parity
from tests.test_gpu_oracle_batched import gradient_views

pytestmark = pytest.mark.gpu

F64 = torch.float64
NAMES = ("means", "log_scales", "quats", "opacity_logits", "sh")


def log(msg):
    print(msg, flush=True)


def to_dev(arrs):
    return [torch.tensor(np.asarray(a, np.float32), device="cuda") for a in arrs]


@pytest.mark.parametrize("seed,tile", [(7, 8), (11, 16)])
def test_3d_filter_images_and_gradients(seed, tile):
    sub, cam, st, target = crops.subcrop_720p(seed)
    st = dataclasses.replace(st, tile_w=tile, tile_h=tile, cost_order=True, tile_cull=True)
    fv = np.random.default_rng(seed).uniform(0.0, 0.04, sub.n).astype(np.float32) ** 2
    arrs = [torch.tensor(a) for a in sub.arrays()]
    ref, info = oracle.render.render(*arrs, sub.sh_degree, cam, st, cull=False, info=True,
                                     filter_var=fv)
    params = to_dev(sub.arrays())
    fvd = torch.tensor(fv, device="cuda")
    frame = htgs.forward(params + [fvd], sub.sh_degree, [cam], st)
    torch.cuda.synchronize()
    assert htgs.read_status(frame.ws)[0] == 0
    stats = parity.check_image(frame.images[0].cpu().numpy(),
                               htgs.state_planes(frame, 0)['core_ids'].cpu().numpy(),
                               ref.numpy(), info, st)
    plain = oracle.render.render(*arrs, sub.sh_degree, cam, st, cull=False).numpy()
    log(f"3D filter seed {seed} tile {tile}: {stats}, filter changes the image by "
        f"{np.abs(plain - ref.numpy()).max():.3f}")
    assert stats['max_err_clean'] < 1e-4 and np.abs(plain - ref.numpy()).max() > 1e-2
    G = np.sign(ref.numpy() - target) / ref.numel()
    G[:, parity.ambiguous_pixels(info, cam.height, cam.width, st)] = 0.0
    ps = [torch.tensor(a, dtype=F64, requires_grad=True) for a in sub.arrays()]
    img = oracle.render.render(*ps, sub.sh_degree, cam, st, cull=False, filter_var=fv)
    (img * torch.tensor(G, dtype=F64)).sum().backward()
    grads = htgs.backward(params + [fvd], frame,
                          [torch.tensor(G, dtype=torch.float32, device="cuda")])
    torch.cuda.synchronize()
    for name, (den, rel, elem) in zip(NAMES, parity.grad_errors(
            [g.cpu().numpy() for g in grads], [p.grad.numpy() for p in ps])):
        log(f"  {name}: |g| {den:.3e}, rel {rel:.2e}, elem {elem:.2e}")
        assert rel <= 1e-3 and elem <= 1e-3, name


@pytest.mark.parametrize("K,tile", [(4, 16), (16, 8)])
def test_baked_inputs_images(K, tile):
    sc, cams, _ = scenes.workload_small()
    cam = cams[0].crop(7, 19, 97, 83)
    q = sc.quats.astype(np.float64)
    baked = scenes.Scene(sc.means, np.exp(sc.log_scales.astype(np.float64)).astype(np.float32),
                         (q / np.linalg.norm(q, axis=1, keepdims=True)).astype(np.float32),
                         (1 / (1 + np.exp(-sc.opacity_logits.astype(np.float64))))
                         .astype(np.float32), sc.sh, sc.sh_degree)
    st = scenes.RenderSettings(K=K, tile_w=tile, tile_h=tile, baked=True, bg=(0.2, 0.1, 0.3))
    frame = htgs.forward(to_dev(baked.arrays()), sc.sh_degree, [cam], st)
    torch.cuda.synchronize()
    assert htgs.read_status(frame.ws)[0] == 0
    ref, info = oracle.render.render_scene(baked, cam, st, info=True)
    stats = parity.check_image(frame.images[0].cpu().numpy(),
                               htgs.state_planes(frame, 0)['core_ids'].cpu().numpy(),
                               ref.numpy(), info, st)
    log(f"baked K={K} tile={tile}: {stats}")
    assert stats['max_err_clean'] < 1e-4


@pytest.mark.parametrize("seed,cull", [(7, False), (13, True)])
def test_densification_sums_match_oracle(seed, cull):
    """Three views in one batched call: the backward adds, per view, |dL_v/dmu|
    times half the mean's distance from the camera to the statistic and 1 to
    the count where the screen box holds a pixel centre."""
    sub, views, st = gradient_views(seed)
    st = dataclasses.replace(st, tile_w=8, tile_h=8, cost_order=True, tile_cull=cull)
    rng = np.random.default_rng(seed + 100)
    Gs = []
    for v in views:
        G = rng.normal(0, 1, (3, v.height, v.width)) / (3 * v.width * v.height)
        _, info = oracle.render.render(*[torch.tensor(a) for a in sub.arrays()], sub.sh_degree,
                                       v, st, cull=False, info=True)
        G[:, parity.ambiguous_pixels(info, v.height, v.width, st)] = 0.0
        Gs.append(G)
    ref_stat, ref_count = oracle.densify.mean_grad_stat(sub.arrays(), sub.sh_degree, views, st, Gs)
    params = to_dev(sub.arrays())
    frame = htgs.forward(params, sub.sh_degree, views, st)
    stat = torch.full((sub.n,), 0.5, device="cuda")
    count = torch.full((sub.n,), 1.0, device="cuda")
    htgs.backward(params, frame, [torch.tensor(G, dtype=torch.float32, device="cuda") for G in Gs],
                  densify=(stat, count))
    torch.cuda.synchronize()
    got_stat = stat.cpu().numpy().astype(np.float64) - 0.5      # added to, not written
    got_count = count.cpu().numpy() - 1.0
    (den, rel, elem), = parity.grad_errors([got_stat], [ref_stat])
    log(f"densify seed {seed} cull {cull}: |stat| {den:.3e}, rel {rel:.2e}, elem {elem:.2e}, "
        f"visible counts {np.bincount(ref_count.astype(int)).tolist()}")
    assert rel <= 1e-3 and elem <= 1e-3
    assert np.array_equal(got_count, ref_count)


def test_opacity_decay_matches_oracle():
    rng = np.random.default_rng(61)
    x = np.concatenate([rng.normal(0, 4, 100_000), [-80.0, -30.0, 0.0, 30.0, 80.0]])
    x = x.astype(np.float32)
    t = torch.tensor(x, device="cuda")
    htgs.opacity_decay(t, 0.9995)
    torch.cuda.synchronize()
    got = t.cpu().numpy().astype(np.float64)
    ref = oracle.densify.opacity_decay(x.astype(np.float64), 0.9995)
    err = np.abs(got - ref) / np.maximum(np.abs(ref), 1.0)
    log(f"opacity decay: max error {err.max():.2e} (relative, or absolute below 1)")
    assert err.max() < 1.2e-7       # one float32 rounding of the float64 result
