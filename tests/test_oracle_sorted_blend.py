"""Pins of the oracle's sorted-blending mode (the paper's "w/o per-pixel HT"
configuration: Sec. 4.3, Table splat_eval; the early stop of Sec. 5).

What fixes the mode independently of its code:
  * a hand-worked pixel (numbers by hand) with and without the early stop;
  * the single isotropic Gaussian closed form;
  * with no early stop and every pixel's fragment depths in the order of
    the mean depths, it is exact depth-sorted alpha blending (Eq.
    alpha_blending, the plain sum of the test helpers);
  * a pair of Gaussians whose per-pixel order differs from their mean
    order: the mean order decides, unlike hybrid transparency;
  * equal mean depths blend in index order; the input order is irrelevant
    otherwise;
  * the stop invariants (T_end >= tau_T; the fragment left out would have
    taken it below tau_T), and tau_T = 1 leaves only the background;
  * tile lists: the instances of the hybrid-transparency lists, each tile
    front to back by the float32 mean depth, then by index;
  * autograd against central differences (no branch change).
"""
import dataclasses

import numpy as np
import pytest
import torch

import oracle
from tests import oracle_helpers as H

F64 = torch.float64


def _frags(sc, cam, st):
    prep = oracle.render.prepare(sc.means, sc.log_scales, sc.quats, sc.opacity_logits, sc.sh,
                                 sc.sh_degree, cam, st, cull=False)
    jj, ii = np.meshgrid(np.arange(cam.height), np.arange(cam.width), indexing='ij')
    xs = torch.tensor(ii.flatten() + 0.5, dtype=F64)
    ys = torch.tensor(jj.flatten() + 0.5, dtype=F64)
    rho2, z, frag, raw, alpha = oracle.render.evaluate(prep, xs, ys, st)
    return prep, z.numpy(), frag.numpy(), alpha.numpy()


def test_hand_worked_pixel_with_and_without_the_stop():
    a = torch.tensor([[0.9, 0.9, 0.5]], dtype=F64)
    f = torch.ones_like(a, dtype=torch.bool)
    col = torch.tensor([[1.0, 0.0, 0.0], [0.0, 1.0, 0.0], [0.0, 0.0, 1.0]], dtype=F64)
    bg = (0.2, 0.4, 0.6)
    order = torch.tensor([0, 1, 2])
    # tau_T = 0.02: after the first fragment T = 0.1; the second would leave
    # 0.01 < 0.02, so it and the third are left out
    C, nb, stop = oracle.blend.sorted_alpha(a, col, f, order, 0.02, bg)
    assert np.allclose(C[0].numpy(), [0.9 + 0.1 * 0.2, 0.1 * 0.4, 0.1 * 0.6], atol=1e-15)
    assert int(nb[0]) == 1 and int(stop[0]) == 1
    # tau_T = 0.004: T goes 1 -> 0.1 -> 0.01 -> 0.005, all three blend
    C, nb, stop = oracle.blend.sorted_alpha(a, col, f, order, 0.004, bg)
    assert np.allclose(C[0].numpy(), [0.9, 0.09, 0.005] + 0.005 * np.array(bg), atol=1e-15)
    assert int(nb[0]) == 3 and int(stop[0]) == -1
    # the order is the one given, not the column order
    C, nb, stop = oracle.blend.sorted_alpha(a, col, f, torch.tensor([2, 0, 1]), 0.004, bg)
    # T: 1 -> 0.5 -> 0.05 -> 0.005
    assert np.allclose(C[0].numpy(), [0.45, 0.045, 0.5] + 0.005 * np.array(bg), atol=1e-15)


def test_single_gaussian_closed_form():
    sigma, z0, o = 0.4, 3.0, 0.8
    sc = H.make_scene([[0.0, 0.0, z0]], [[np.log(sigma)] * 3], [[1, 0, 0, 0]],
                      [np.log(o / (1 - o))], [[0.9, 0.3, 0.1]])
    cam = H.simple_camera(16, 16, 20.0)
    bg = np.array([0.1, 0.5, 0.2])
    st = H.settings(sorted_blend=True, bg=tuple(bg), tau_T=1e-4)
    img = oracle.render.render_scene(sc, cam, st, cull=False).numpy()
    o32 = float(1.0 / (1.0 + np.exp(-np.float64(np.float32(np.log(o / (1 - o)))))))
    s32 = float(np.exp(np.float64(np.float32(np.log(sigma)))))
    rho_c = 2 * np.log(o32 * 255.0)
    for j in range(16):
        for i in range(16):
            u = (i + 0.5 - cam.cx) / cam.fx
            v = (j + 0.5 - cam.cy) / cam.fy
            r2 = z0 * z0 * (u * u + v * v) / ((1 + u * u + v * v) * s32 * s32)
            a = min(0.99, o32 * np.exp(-0.5 * r2)) if r2 <= rho_c else 0.0
            ref = a * np.array([0.9, 0.3, 0.1], np.float32) + (1 - a) * bg
            assert np.abs(img[:, j, i] - ref).max() < 1e-6


def test_axis_aligned_isotropic_stack_is_exact_sorted_blending():
    """Isotropic Gaussians with their means on the optical axis: along every
    ray the maximum point of each lies at depth mu_z r_z^2, so all pixels
    see them in mean-depth order. Without the stop, sorted blending is
    then Eq. alpha_blending at every pixel."""
    rng = np.random.default_rng(5)
    n = 9
    means = np.stack([np.zeros(n), np.zeros(n), rng.permutation(np.linspace(2.0, 6.0, n))], 1)
    ls = np.repeat(rng.normal(-1.0, 0.3, (n, 1)), 3, 1)
    sc = H.make_scene(means, ls, rng.normal(0, 1, (n, 4)), rng.normal(1.0, 1.0, n),
                      rng.uniform(0.05, 0.95, (n, 3)))
    cam = H.simple_camera(18, 18, 22.0)
    bg = (0.3, 0.2, 0.7)
    st = H.settings(sorted_blend=True, tau_T=0.0, bg=bg)
    img = oracle.render.render_scene(sc, cam, st, cull=False).numpy()
    prep, z, frag, alpha = _frags(sc, cam, st)
    col = prep.colour.numpy()
    deepest = 0
    for p in range(cam.width * cam.height):
        ids = np.nonzero(frag[p])[0]
        deepest = max(deepest, len(ids))
        ref = H.sorted_blend(alpha[p, ids], col[ids], z[p, ids], bg)
        j, i = divmod(p, cam.width)
        assert np.abs(img[:, j, i] - ref).max() < 1e-14
    assert deepest >= 5


def test_mean_order_decides_not_the_pixel_depth():
    """A thin disc tilted towards the camera whose mean lies behind a small
    ball: at pixels where the disc's surface is in front of the ball,
    hybrid transparency (per-pixel depth) puts the disc first, sorted
    blending still the ball (its mean is nearer)."""
    ang = np.radians(70.0)
    q_disc = [np.cos(ang / 2), np.sin(ang / 2), 0.0, 0.0]       # about the x axis
    sc = H.make_scene([[0.0, 0.0, 3.0], [0.0, 0.35, 3.2]],
                      [[np.log(0.12)] * 3, [np.log(0.6), np.log(0.6), np.log(0.005)]],
                      [[1, 0, 0, 0], q_disc], [1.5, 1.5],
                      [[0.9, 0.1, 0.1], [0.1, 0.1, 0.9]])
    cam = H.simple_camera(24, 24, 30.0)
    bg = (0.0, 0.0, 0.0)
    st_s = H.settings(sorted_blend=True, tau_T=0.0, bg=bg)
    img = oracle.render.render_scene(sc, cam, st_s, cull=False).numpy()
    prep, z, frag, alpha = _frags(sc, cam, st_s)
    col = prep.colour.numpy()
    swapped = 0
    for p in range(cam.width * cam.height):
        if not (frag[p, 0] and frag[p, 1]):
            continue
        j, i = divmod(p, cam.width)
        ball_first = alpha[p, 0] * col[0] + (1 - alpha[p, 0]) * alpha[p, 1] * col[1]
        assert np.abs(img[:, j, i] - ball_first).max() < 1e-14
        if z[p, 1] < z[p, 0]:
            swapped += 1
    assert swapped >= 3   # the disc is in front at several pixels


def test_equal_mean_depths_blend_in_index_order():
    cols = [[0.9, 0.1, 0.1], [0.1, 0.9, 0.1]]
    sc = H.make_scene([[0.02, 0.0, 3.0], [-0.02, 0.0, 3.0]], [[np.log(0.3)] * 3] * 2,
                      [[1, 0, 0, 0]] * 2, [0.5, 2.0], cols)
    cam = H.simple_camera(8, 8, 12.0)
    st = H.settings(sorted_blend=True, tau_T=0.0)
    img = oracle.render.render_scene(sc, cam, st, cull=False).numpy()
    prep, z, frag, alpha = _frags(sc, cam, st)
    col = prep.colour.numpy()
    for p in range(64):
        j, i = divmod(p, 8)
        ref = alpha[p, 0] * col[0] + (1 - alpha[p, 0]) * alpha[p, 1] * col[1]
        assert np.abs(img[:, j, i] - ref).max() < 1e-14
    # swapping the two Gaussians' indices swaps which one is in front
    sc2 = H.make_scene([[-0.02, 0.0, 3.0], [0.02, 0.0, 3.0]], [[np.log(0.3)] * 3] * 2,
                       [[1, 0, 0, 0]] * 2, [2.0, 0.5], cols[::-1])
    img2 = oracle.render.render_scene(sc2, cam, st, cull=False).numpy()
    assert np.abs(img2 - img).max() > 1e-3


def test_input_order_is_irrelevant_away_from_ties():
    sc = H.tiny_random_scene(14, seed=21)
    cam = H.simple_camera(16, 16, 25.0)
    st = H.settings(sorted_blend=True, tau_T=1e-3, bg=(0.2, 0.3, 0.4))
    img = oracle.render.render_scene(sc, cam, st, cull=False).numpy()
    perm = np.random.default_rng(2).permutation(sc.n)
    img2 = oracle.render.render_scene(sc.subset(perm), cam, st, cull=False).numpy()
    assert np.abs(img - img2).max() < 1e-14


def test_stop_invariants_and_full_stop():
    sc = H.tiny_random_scene(24, seed=8, log_scale=-1.2)
    sc.opacity_logits[:] = 4.0   # dense and opaque: stops happen
    cam = H.simple_camera(16, 16, 25.0)
    tau = 0.02
    st = H.settings(sorted_blend=True, tau_T=tau)
    prep, z, frag, alpha = _frags(sc, cam, st)
    order = oracle.blend.depth_order(oracle.splat.mean_view_depth32(sc.means, cam)
                                     [prep.idx.numpy()])
    C, nb, stop = oracle.blend.sorted_alpha(torch.tensor(alpha), prep.colour, torch.tensor(frag),
                                            order, tau, st.bg)
    n_stops = 0
    for p in range(cam.width * cam.height):
        seq = [g for g in order.tolist() if frag[p, g]]
        T = 1.0
        for g in seq[:int(nb[p])]:
            T *= 1.0 - alpha[p, g]
        assert T >= tau
        if int(stop[p]) >= 0:
            n_stops += 1
            g = seq[int(nb[p])]
            assert g == int(stop[p]) and T * (1.0 - alpha[p, g]) < tau
        else:
            assert int(nb[p]) == len(seq)
    assert n_stops >= 10
    # tau_T = 1: any fragment would take T below it; only the background
    st1 = H.settings(sorted_blend=True, tau_T=1.0, bg=(0.25, 0.5, 0.75))
    img = oracle.render.render_scene(sc, cam, st1, cull=False).numpy()
    assert np.abs(img - np.array(st1.bg)[:, None, None]).max() == 0.0


def test_tile_lists_are_depth_ordered_ht_instances():
    sc = H.tiny_random_scene(40, seed=13, spread=1.2)
    cam = H.simple_camera(40, 32, 25.0)
    st = H.settings(tile_w=8, tile_h=8)
    ref = oracle.bins.tile_lists(sc.means, sc.log_scales, sc.quats, sc.opacity_logits, cam, st)
    srt = oracle.bins.tile_lists(sc.means, sc.log_scales, sc.quats, sc.opacity_logits, cam,
                                 dataclasses.replace(st, sorted_blend=True))
    assert np.array_equal(srt['keys'], ref['keys'])
    assert sorted(zip(srt['keys'], srt['values'])) == sorted(zip(ref['keys'], ref['values']))
    # the view depth of the means, by the pinhole model (this camera: z + 0)
    zt = sc.means[:, 2].astype(np.float32)
    assert np.array_equal(srt['depth32'], zt)
    for t in np.unique(srt['keys']):
        v = srt['values'][srt['keys'] == t]
        pairs = list(zip(zt[v].tolist(), v.tolist()))
        assert pairs == sorted(pairs)


def test_sorted_gradient_matches_central_differences():
    sc = H.tiny_random_scene(6, seed=31, log_scale=-1.3)
    cam = H.simple_camera(12, 12, 18.0)
    st = H.settings(sorted_blend=True, tau_T=0.05, bg=(0.1, 0.2, 0.3))
    G = torch.tensor(np.random.default_rng(1).normal(0, 1, (3, 12, 12)), dtype=F64)
    arrs = [torch.tensor(a, dtype=F64) for a in sc.arrays()]

    def loss(ps):
        return float((oracle.render.render(*ps, sc.sh_degree, cam, st, cull=False) * G).sum())

    def branches(ps):
        _, info = oracle.render.render(*ps, sc.sh_degree, cam, st, cull=False, info=True)
        fr = info['frags']
        return (info['core'].numpy().tobytes(), fr['frag'].tobytes(),
                (fr['raw'] >= st.alpha_max).tobytes())

    ps = [a.clone().requires_grad_(True) for a in arrs]
    (oracle.render.render(*ps, sc.sh_degree, cam, st, cull=False) * G).sum().backward()
    base = branches(arrs)
    h = 1e-6
    checked = 0
    rng = np.random.default_rng(4)
    for ti, a in enumerate(arrs):
        flat = a.flatten()
        for k in rng.choice(flat.numel(), min(12, flat.numel()), replace=False):
            plus = [x.clone() for x in arrs]
            minus = [x.clone() for x in arrs]
            plus[ti].view(-1)[k] += h
            minus[ti].view(-1)[k] -= h
            if branches(plus) != base or branches(minus) != base:
                continue
            fd = (loss(plus) - loss(minus)) / (2 * h)
            g = float(ps[ti].grad.view(-1)[k])
            assert abs(fd - g) <= 1e-6 * max(1.0, abs(g)), (ti, k, fd, g)
            checked += 1
    assert checked >= 40
