"""Pins of the oracle's 3D smoothing filter and baked inputs (CPU only).

The filter (Mip-Splatting, used in Sec. 4.2 of the paper in place of a
screen-space filter) replaces each Gaussian's peak-normalised density
o exp(-x^T Sigma^-1 x / 2) by its convolution with a unit-mass isotropic
Gaussian of variance f. The pins compute that convolution by numerical
quadrature, independently of the oracle's closed form (which adds f to the
squared scales and scales o by sqrt(det Sigma / det Sigma')). Baked inputs
(frame-rate appendix) hold the activations' results and must render the
same image as the raw parameters."""
import math

import numpy as np
import pytest
import torch
from scipy import integrate

import oracle
from tests import oracle_helpers as H

F64 = torch.float64


def _convolved_density(o, s, R, f, x):
    """(o exp(-y^T S^-2 y / 2) * N(0, f I))(x), y the splat frame: the
    isotropic kernel keeps its form in the splat's own (rotated) frame, where
    the integral factorises into three 1D integrals."""
    y = R.T @ x
    val = o
    for k in range(3):
        def integrand(t, k=k):
            return (math.exp(-0.5 * t * t / (s[k] * s[k])) *
                    math.exp(-0.5 * (y[k] - t) ** 2 / f) / math.sqrt(2 * math.pi * f))
        w = max(s[k], math.sqrt(f))
        lo, hi = min(0.0, y[k]) - 14 * w, max(0.0, y[k]) + 14 * w
        val *= integrate.quad(integrand, lo, hi, points=sorted({0.0, float(y[k])}),
                              epsabs=1e-15, epsrel=1e-13, limit=400)[0]
    return val


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_filter_equals_convolution_by_quadrature(seed):
    rng = np.random.default_rng(seed)
    ls = rng.normal(-1.5, 0.6, 3)
    q = rng.normal(0, 1, 4)
    logit = rng.normal(0, 1)
    f = float(rng.uniform(0.01, 0.2)) ** 2
    s_f, R, o_f = oracle.splat.activations(torch.tensor(ls[None]), torch.tensor(q[None]),
                                           torch.tensor([logit], dtype=F64),
                                           filter_var=np.array([f]))
    s_f, R, o_f = s_f[0].numpy(), R[0].numpy(), float(o_f[0])
    s, o = np.exp(ls), 1 / (1 + math.exp(-logit))
    for _ in range(6):
        x = rng.normal(0, 1, 3) * s_f
        y = R.T @ x
        closed = o_f * math.exp(-0.5 * float(np.sum((y / s_f) ** 2)))
        ref = _convolved_density(o, s, R, f, x)
        assert abs(closed - ref) <= 1e-9 * max(ref, 1e-30) + 1e-13, (closed, ref)


def test_zero_filter_variance_changes_nothing():
    sc = H.tiny_random_scene(12, seed=41)
    cam = H.simple_camera(16, 16, 25.0)
    st = H.settings(K=4, bg=(0.1, 0.2, 0.3))
    a = oracle.render.render_scene(sc, cam, st, cull=False).numpy()
    b = oracle.render.render_scene(sc, cam, st, cull=False,
                                   filter_var=np.zeros(sc.n)).numpy()
    assert np.abs(a - b).max() < 1e-15


def test_filter_widens_and_dims_every_splat():
    sc = H.tiny_random_scene(12, seed=42)
    f = np.full(sc.n, 0.02 ** 2)
    s0, _, o0 = oracle.splat.activations(torch.tensor(sc.log_scales, dtype=F64),
                                         torch.tensor(sc.quats, dtype=F64),
                                         torch.tensor(sc.opacity_logits, dtype=F64))
    s1, _, o1 = oracle.splat.activations(torch.tensor(sc.log_scales, dtype=F64),
                                         torch.tensor(sc.quats, dtype=F64),
                                         torch.tensor(sc.opacity_logits, dtype=F64), filter_var=f)
    assert (s1 > s0).all() and (o1 < o0).all()
    # the filtered splat's total mass o' (2 pi)^1.5 prod s' equals the unfiltered one's
    m0 = o0 * torch.prod(s0, 1)
    m1 = o1 * torch.prod(s1, 1)
    assert torch.allclose(m0, m1, rtol=1e-13, atol=0)


def test_filtered_zero_axis_splat_vanishes():
    """A zero scale axis has no volume: convolved with a finite filter its
    peak opacity drops to zero, and the splat is culled."""
    sc = H.tiny_random_scene(4, seed=43)
    sc.log_scales[0, 1] = -np.inf
    _, _, o = oracle.splat.activations(torch.tensor(sc.log_scales, dtype=F64),
                                       torch.tensor(sc.quats, dtype=F64),
                                       torch.tensor(sc.opacity_logits, dtype=F64),
                                       filter_var=np.full(sc.n, 1e-4))
    assert float(o[0]) == 0.0 and (o[1:] > 0).all()


def test_baked_inputs_render_the_same_image():
    sc = H.tiny_random_scene(14, seed=44)
    cam = H.simple_camera(18, 18, 25.0)
    st = H.settings(K=4, bg=(0.3, 0.1, 0.2))
    q = sc.quats.astype(np.float64)
    baked = [sc.means, np.exp(sc.log_scales.astype(np.float64)),
             q / np.linalg.norm(q, axis=1, keepdims=True),
             1 / (1 + np.exp(-sc.opacity_logits.astype(np.float64))), sc.sh]
    a = oracle.render.render_scene(sc, cam, st, cull=False).numpy()
    b = oracle.render.render(*baked, sc.sh_degree, cam, H.settings(K=4, bg=(0.3, 0.1, 0.2),
                                                                   baked=True), cull=False).numpy()
    assert np.abs(a - b).max() < 1e-13


def test_filter_gradient_matches_central_differences():
    """Through the filter the scales and opacity logits still get their
    exact float64 derivative (autograd against central differences)."""
    sc = H.tiny_random_scene(6, seed=45, spread=0.4)
    cam = H.simple_camera(12, 12, 18.0)
    st = H.settings(K=3, bg=(0.2, 0.3, 0.1))
    f = np.random.default_rng(45).uniform(0.0, 0.05, sc.n) ** 2
    base = [torch.tensor(x, dtype=F64) for x in sc.arrays()]
    ps = [b.clone().requires_grad_(True) for b in base]
    img = oracle.render.render(*ps, sc.sh_degree, cam, st, cull=False, filter_var=f)
    G = torch.tensor(np.random.default_rng(1).normal(0, 1, img.shape), dtype=F64)
    (img * G).sum().backward()
    h = 1e-6
    worst = 0.0
    for t in (1, 3):            # log-scales, opacity logits
        gmax = float(ps[t].grad.abs().max())
        for off in range(base[t].numel()):
            vals = []
            for sgn in (1, -1):
                pp = [b.clone() for b in base]
                pp[t].view(-1)[off] += sgn * h
                vals.append(float((oracle.render.render(*pp, sc.sh_degree, cam, st, cull=False,
                                                        filter_var=f) * G).sum()))
            fd = (vals[0] - vals[1]) / (2 * h)
            an = float(ps[t].grad.view(-1)[off])
            worst = max(worst, abs(fd - an) / gmax)
    assert worst < 1e-5, worst
