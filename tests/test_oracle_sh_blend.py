"""Pins for the oracle's SH colour (Sec. 3.1) and hybrid-transparency
composite (Sec. 3.3)."""
import math

import numpy as np
import pytest
import scipy.special
import torch

import oracle

from tests import oracle_helpers as H

F64 = torch.float64


def _real_sh_scipy(l, m, theta, phi):
    """Orthonormal real SH without the Condon-Shortley phase, from scipy's
    complex Y_l^m (which includes that phase)."""
    if m == 0:
        return scipy.special.sph_harm_y(l, 0, theta, phi).real
    Y = scipy.special.sph_harm_y(l, abs(m), theta, phi)
    sgn = (-1) ** abs(m)
    return math.sqrt(2.0) * sgn * (Y.imag if m < 0 else Y.real)


def test_sh_basis_matches_scipy_definition():
    rng = np.random.default_rng(0)
    d = rng.normal(0, 1, (200, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    theta = np.arccos(d[:, 2])
    phi = np.arctan2(d[:, 1], d[:, 0])
    Y = oracle.sh.basis(torch.tensor(d), 3).numpy()
    for l in range(4):
        for m in range(-l, l + 1):
            ref = _real_sh_scipy(l, m, theta, phi)
            np.testing.assert_allclose(Y[:, l * l + l + m], ref, atol=1e-13)


def test_sh_basis_orthonormal_by_quadrature():
    x, w = np.polynomial.legendre.leggauss(24)          # cos(theta) nodes
    phi = (np.arange(48) + 0.5) * 2 * math.pi / 48
    ct, ph = np.meshgrid(x, phi, indexing='ij')
    st = np.sqrt(1 - ct ** 2)
    d = np.stack([st * np.cos(ph), st * np.sin(ph), ct], -1).reshape(-1, 3)
    wt = (w[:, None] * np.full(48, 2 * math.pi / 48)[None, :]).reshape(-1)
    Y = oracle.sh.basis(torch.tensor(d), 3).numpy()
    G = (Y * wt[:, None]).T @ Y
    np.testing.assert_allclose(G, np.eye(16), atol=1e-12)


def test_sh_dc_colour_is_view_independent_and_direction_convention():
    sh = torch.zeros(1, 16, 3, dtype=F64)
    sh[0, 0] = torch.tensor([0.3, -0.2, 0.9])
    mu = torch.tensor([[0.5, -1.0, 4.0]], dtype=F64)
    c1 = oracle.sh.colour(sh, mu, torch.tensor([0.0, 0.0, 0.0], dtype=F64), 3)
    c2 = oracle.sh.colour(sh, mu, torch.tensor([7.0, 2.0, -3.0], dtype=F64), 3)
    assert torch.allclose(c1, c2, atol=0, rtol=0)
    ref = 0.5 / math.sqrt(math.pi) * torch.tensor([0.3, -0.2, 0.9]) + 0.5
    assert torch.allclose(c1[0], ref.to(F64).clamp(min=0))
    # direction runs from the camera centre to the mean: a pure z-band
    # coefficient brightens a Gaussian straight ahead along +z
    sh = torch.zeros(1, 4, 3, dtype=F64)
    sh[0, 2] = 0.4
    k = math.sqrt(3 / (4 * math.pi)) * 0.4
    fwd = oracle.sh.colour(sh, torch.tensor([[0.0, 0.0, 5.0]], dtype=F64),
                           torch.zeros(3, dtype=F64), 1)
    back = oracle.sh.colour(sh, torch.tensor([[0.0, 0.0, 5.0]], dtype=F64),
                            torch.tensor([0.0, 0.0, 9.0], dtype=F64), 1)
    assert abs(float(fwd[0, 0]) - (0.5 + k)) < 1e-15
    assert abs(float(back[0, 0]) - (0.5 - k)) < 1e-15


def test_sh_clamps_at_zero():
    sh = torch.zeros(1, 1, 3, dtype=F64)
    sh[0, 0] = torch.tensor([-5.0, 0.0, 5.0])
    c = oracle.sh.colour(sh, torch.tensor([[0.0, 0.0, 1.0]], dtype=F64), torch.zeros(3, dtype=F64), 0)
    assert float(c[0, 0]) == 0.0 and float(c[0, 1]) == 0.5


def _pixel_fragments(sc, cam, st):
    prep = oracle.render.prepare(sc.means, sc.log_scales, sc.quats, sc.opacity_logits, sc.sh,
                                 sc.sh_degree, cam, st, cull=False)
    jj, ii = np.meshgrid(np.arange(cam.height), np.arange(cam.width), indexing='ij')
    xs = torch.tensor(ii.flatten() + 0.5, dtype=F64)
    ys = torch.tensor(jj.flatten() + 0.5, dtype=F64)
    rho2, z, frag, raw, alpha = oracle.render.evaluate(prep, xs, ys, st)
    return prep, z.numpy(), frag.numpy(), alpha.numpy()


def test_ht_with_large_core_equals_exact_sorted_blending():
    sc = H.tiny_random_scene(14, seed=4)
    cam = H.simple_camera(20, 20, 30.0)
    bg = (0.15, 0.6, 0.35)
    st = H.settings(K=32, tau_core=0.0, bg=bg)
    img = oracle.render.render_scene(sc, cam, st, cull=False).numpy()
    prep, z, frag, alpha = _pixel_fragments(sc, cam, st)
    col = prep.colour.numpy()
    n_frag_max = 0
    for p in range(cam.width * cam.height):
        ids = np.nonzero(frag[p])[0]
        n_frag_max = max(n_frag_max, len(ids))
        ref = H.sorted_blend(alpha[p, ids], col[ids], z[p, ids], bg)
        j, i = divmod(p, cam.width)
        assert np.abs(img[:, j, i] - ref).max() < 1e-14
    assert n_frag_max >= 5  # the scene does overlap


@pytest.mark.parametrize("K", [0, 1, 3, 8])
def test_ht_equal_colour_tail_is_exact(K):
    sc = H.tiny_random_scene(14, seed=6)
    sc.sh[:] = sc.sh[:1]        # every Gaussian has the same colour
    cam = H.simple_camera(16, 16, 25.0)
    bg = (0.7, 0.2, 0.4)
    st = H.settings(K=K, bg=bg)
    img = oracle.render.render_scene(sc, cam, st, cull=False).numpy()
    prep, z, frag, alpha = _pixel_fragments(sc, cam, st)
    col = prep.colour.numpy()
    for p in range(cam.width * cam.height):
        ids = np.nonzero(frag[p])[0]
        ref = H.sorted_blend(alpha[p, ids], col[ids], z[p, ids], bg)
        j, i = divmod(p, cam.width)
        assert np.abs(img[:, j, i] - ref).max() < 1e-14


def test_ht_k0_is_pure_tail_formula():
    sc = H.tiny_random_scene(10, seed=11)
    cam = H.simple_camera(16, 16, 25.0)
    bg = np.array([0.3, 0.1, 0.8])
    st = H.settings(K=0, bg=tuple(bg))
    img = oracle.render.render_scene(sc, cam, st, cull=False).numpy()
    prep, z, frag, alpha = _pixel_fragments(sc, cam, st)
    col = prep.colour.numpy()
    for p in range(cam.width * cam.height):
        ids = np.nonzero(frag[p])[0]
        a = alpha[p, ids]
        A = a.sum()
        Pt = np.prod(1 - a)
        ref = Pt * bg + ((1 - Pt) * (a[:, None] * col[ids]).sum(0) / A if A > 0 else 0)
        j, i = divmod(p, cam.width)
        assert np.abs(img[:, j, i] - ref).max() < 1e-14


def test_ht_core_and_tail_split_by_hand():
    """Three fragments at one pixel with K = 1: the nearest eligible one is
    the core, the other two (one below tau_K) form the tail."""
    a = torch.tensor([0.5, 0.03, 0.6], dtype=F64)
    z = torch.tensor([3.0, 1.0, 2.0], dtype=F64)
    c = torch.tensor([[1.0, 0, 0], [0, 1.0, 0], [0, 0, 1.0]], dtype=F64)
    frag = torch.ones(1, 3, dtype=torch.bool)
    bg = torch.tensor([0.1, 0.2, 0.3], dtype=F64)
    C, core = oracle.blend.hybrid(a[None], c, z[None], frag, 1, 0.05, bg)
    # core: index 2 (depth 2, alpha 0.6); index 1 is nearer but below tau_K
    assert core.tolist() == [[2]]
    T2 = 0.4
    At = 0.5 + 0.03
    ctail = (0.5 * c[0] + 0.03 * c[1]) / At
    Pt = 0.5 * 0.97
    ref = 0.6 * c[2] + T2 * ((1 - Pt) * ctail + Pt * bg)
    assert torch.allclose(C[0], ref, atol=1e-15, rtol=0)
    ref2 = oracle.blend.composite_pixel([a[2]], [c[2]], [a[0], a[1]], [c[0], c[1]], bg)
    assert torch.allclose(ref2, ref, atol=1e-15, rtol=0)


def test_ht_depth_ties_break_by_index():
    a = torch.tensor([[0.4, 0.7]], dtype=F64)
    z = torch.tensor([[2.0, 2.0]], dtype=F64)
    c = torch.eye(3, dtype=F64)[:2]
    _, core = oracle.blend.hybrid(a, c, z, torch.ones(1, 2, dtype=torch.bool), 1, 0.05,
                                  torch.zeros(3, dtype=F64))
    assert core.tolist() == [[0]]


def test_ht_permutation_invariance():
    sc = H.tiny_random_scene(16, seed=12)
    cam = H.simple_camera(16, 16, 25.0)
    st = H.settings(K=3, bg=(0.2, 0.2, 0.2))
    ref = oracle.render.render_scene(sc, cam, st, cull=False).numpy()
    perm = np.random.default_rng(0).permutation(sc.n)
    img = oracle.render.render_scene(sc.subset(perm), cam, st, cull=False).numpy()
    assert np.abs(img - ref).max() < 1e-14


def test_degenerate_splats_finite_image_and_gradients():
    sc = H.tiny_random_scene(12, seed=13)
    sc.log_scales[:4, 0] = -np.inf
    sc.log_scales[4:6, 1] = np.float32(math.log(1e-7))
    sc.log_scales[6, :2] = -np.inf
    cam = H.simple_camera(16, 16, 25.0)
    st = H.settings(K=4)
    params = [torch.tensor(x, dtype=F64, requires_grad=True) for x in sc.arrays()]
    img = oracle.render.render(*params, sc.sh_degree, cam, st, cull=False)
    assert torch.isfinite(img).all()
    (img * torch.linspace(-1, 1, img.numel(), dtype=F64).reshape(img.shape)).sum().backward()
    for p in params:
        assert torch.isfinite(p.grad).all()
    # the flat splats do contribute fragments
    prep, z, frag, alpha = _pixel_fragments(sc, cam, st)
    kept = prep.idx.numpy()
    assert frag[:, np.isin(kept, [0, 1, 2, 3])].any()





# ---------------------------------------------------------------------------
# Inference without the tail (Sec. 4.3, Table ablations)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("K", [1, 3, 8])
def test_no_tail_is_sorted_blending_of_the_core_alone(K):
    """Per pixel: the K nearest fragments with alpha >= tau_K (ties by
    index), alpha-blended in depth order over the background; every other
    fragment is ignored."""
    sc = H.tiny_random_scene(16, seed=31)
    cam = H.simple_camera(18, 18, 28.0)
    bg = (0.25, 0.5, 0.9)
    st = H.settings(K=K, bg=bg, no_tail=True)
    img = oracle.render.render_scene(sc, cam, st, cull=False).numpy()
    full = oracle.render.render_scene(sc, cam, H.settings(K=K, bg=bg), cull=False).numpy()
    prep, z, frag, alpha = _pixel_fragments(sc, cam, st)
    col = prep.colour.numpy()
    n_diff = 0
    for p in range(cam.width * cam.height):
        ids = [int(i) for i in np.nonzero(frag[p] & (alpha[p] >= st.tau_core))[0]]
        core = sorted(ids, key=lambda i: (z[p, i], int(prep.idx[i])))[:K]
        ref = H.sorted_blend(alpha[p, core], col[core], z[p, core], bg)
        j, i = divmod(p, cam.width)
        assert np.abs(img[:, j, i] - ref).max() < 1e-14
        n_diff += int(np.abs(img[:, j, i] - full[:, j, i]).max() > 1e-6)
    assert n_diff > 10     # the tail does matter somewhere in this scene


def test_no_tail_equals_hybrid_when_the_tail_is_empty():
    """K at least the fragment count and tau_K = 0: the core holds every
    fragment, the tail is empty, so both modes give exact sorted blending."""
    sc = H.tiny_random_scene(12, seed=32)
    cam = H.simple_camera(16, 16, 25.0)
    st = H.settings(K=32, tau_core=0.0, bg=(0.1, 0.2, 0.3))
    a = oracle.render.render_scene(sc, cam, st, cull=False).numpy()
    b = oracle.render.render_scene(sc, cam, H.settings(K=32, tau_core=0.0, bg=(0.1, 0.2, 0.3),
                                                       no_tail=True), cull=False).numpy()
    assert np.abs(a - b).max() < 1e-14


def test_no_tail_with_empty_core_is_background():
    sc = H.tiny_random_scene(12, seed=33)
    cam = H.simple_camera(16, 16, 25.0)
    bg = (0.4, 0.3, 0.2)
    img = oracle.render.render_scene(sc, cam, H.settings(K=0, bg=bg, no_tail=True),
                                     cull=False).numpy()
    assert np.abs(img - np.array(bg)[:, None, None]).max() == 0.0
