"""Pins of the oracle's training-side quantities (Sec. 4.2), CPU only.

* Densification statistic: per view, the norm of the mean's gradient
  (here by central differences of the float64 render, not autograd) times
  half the mean's distance from the eye the camera was built at; the view
  count from hand-placed Gaussians (in view, behind the camera, outside the
  frustum).
* Opacity decay: an independent rearrangement of logit(lambda sigmoid(x)),
  its limits, and lambda^k for k repeated decays."""
import math

import numpy as np
import torch

import oracle
from paper_2410_08129_amd import scenes
from tests import oracle_helpers as H

F64 = torch.float64


def test_mean_grad_stat_is_scaled_mean_gradient_norm():
    sc = H.tiny_random_scene(5, seed=51, spread=0.35)
    eyes = [(0.0, 0.0, 0.0), (0.4, -0.3, 0.2)]
    cams = [scenes.look_at(e, (0.0, 0.0, 4.0), (0, -1, 0), 40.0, 14, 12) for e in eyes]
    st = H.settings(K=2, bg=(0.1, 0.1, 0.1))
    rng = np.random.default_rng(5)
    Gs = [rng.normal(0, 1, (3, c.height, c.width)) for c in cams]
    stat, count = oracle.densify.mean_grad_stat(sc.arrays(), sc.sh_degree, cams, st, Gs)
    ref = np.zeros(sc.n)
    h = 1e-6
    for cam, G, eye in zip(cams, Gs, eyes):
        base = [np.asarray(a, np.float64) for a in sc.arrays()]
        grad = np.zeros((sc.n, 3))
        for g in range(sc.n):
            for k in range(3):
                vals = []
                for sgn in (1, -1):
                    arr = [b.copy() for b in base]
                    arr[0][g, k] += sgn * h
                    img = oracle.render.render(*[torch.tensor(a) for a in arr], sc.sh_degree, cam,
                                               st, cull=False)
                    vals.append(float((img.numpy() * G).sum()))
                grad[g, k] = (vals[0] - vals[1]) / (2 * h)
        dist = np.linalg.norm(base[0] - np.asarray(eye), axis=1)
        ref += np.linalg.norm(grad, axis=1) * dist / 2
    assert np.abs(stat - ref).max() <= 1e-6 * max(np.abs(ref).max(), 1e-30)
    assert (stat > 0).sum() >= 3
    assert count.tolist() == [2.0] * sc.n


def test_visible_count_by_hand():
    # a: in front of both cameras; b: behind the second camera; c: far
    # outside the first camera's frustum
    sc = H.make_scene([[0.0, 0.0, 3.0], [0.0, 0.0, -3.0], [40.0, 0.0, 3.0]],
                      [[-2.0] * 3] * 3, [[1, 0, 0, 0]] * 3, [2.0] * 3,
                      colours=[[0.5, 0.5, 0.5]] * 3)
    cams = [scenes.look_at((0, 0, 0), (0, 0, 1), (0, -1, 0), 50.0, 32, 32),
            scenes.look_at((0, 0, -6), (0, 0, 0), (0, -1, 0), 50.0, 32, 32)]
    st = H.settings(K=2)
    Gs = [np.ones((3, 32, 32)) for _ in cams]
    _, count = oracle.densify.mean_grad_stat(sc.arrays(), sc.sh_degree, cams, st, Gs)
    assert count.tolist() == [2.0, 1.0, 0.0]


def test_opacity_decay_rearrangement_and_limits():
    lam = 0.9995
    x = np.concatenate([np.linspace(-30, 30, 121), [-700.0, 700.0]])
    y = oracle.densify.opacity_decay(x, lam)
    alt = np.where(x >= 0, math.log(lam) - np.log(np.exp(-np.minimum(x, 700)) + 1 - lam),
                   x + math.log(lam) - np.log1p((1 - lam) * np.exp(np.minimum(x, 0))))
    fin = np.abs(x) <= 30
    assert np.abs(y[fin] - alt[fin]).max() < 1e-12
    assert (np.diff(y[:121]) > 0).all() and (y[:121] < x[:121]).all()
    assert abs(y[-1] - math.log(lam / (1 - lam))) < 1e-9          # opacity saturates at lambda
    assert abs(y[-2] - (-700.0 + math.log(lam))) < 1e-9           # tiny opacities scale by lambda
    z = x[:121]
    for _ in range(5):
        z = oracle.densify.opacity_decay(z, lam)
    assert np.abs(oracle.densify.opacity_decay(x[:121], lam ** 5) - z).max() < 1e-9
