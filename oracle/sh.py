"""View-dependent colour from real spherical harmonics (paper Sec. 3.1: the
colour model is that of 3DGS, SH up to degree 3, 48 coefficients).

Basis: the orthonormal real spherical harmonics without the Condon-Shortley
phase, Y_{l,m} for l <= 3, coefficient index l*l + l + m, written here as
polynomials of the unit direction (x, y, z). Colour per channel is
max(0, sum_lm k_lm Y_lm(dir) + 0.5) with dir the unit vector from the camera
centre to the Gaussian's mean (3DGS convention).
"""
from __future__ import annotations

import math

import torch

_PI = math.pi


def basis(dirs, degree):
    """Real SH basis at unit directions ``dirs`` [n,3] -> [n,(degree+1)^2]."""
    x, y, z = dirs.unbind(-1)
    out = [torch.full_like(x, 0.5 * math.sqrt(1.0 / _PI))]
    if degree >= 1:
        c1 = math.sqrt(3.0 / (4.0 * _PI))
        out += [c1 * y, c1 * z, c1 * x]
    if degree >= 2:
        c2 = 0.5 * math.sqrt(15.0 / _PI)
        out += [c2 * x * y,
                c2 * y * z,
                0.25 * math.sqrt(5.0 / _PI) * (3.0 * z * z - 1.0),
                c2 * x * z,
                0.25 * math.sqrt(15.0 / _PI) * (x * x - y * y)]
    if degree >= 3:
        a = 0.25 * math.sqrt(35.0 / (2.0 * _PI))
        b = 0.5 * math.sqrt(105.0 / _PI)
        c = 0.25 * math.sqrt(21.0 / (2.0 * _PI))
        d = 0.25 * math.sqrt(7.0 / _PI)
        e = 0.25 * math.sqrt(105.0 / _PI)
        out += [a * y * (3.0 * x * x - y * y),
                b * x * y * z,
                c * y * (5.0 * z * z - 1.0),
                d * z * (5.0 * z * z - 3.0),
                c * x * (5.0 * z * z - 1.0),
                e * z * (x * x - y * y),
                a * x * (x * x - 3.0 * y * y)]
    return torch.stack(out, dim=-1)


def colour(sh, means, cam_center, degree):
    """RGB [n,3] of each Gaussian seen from ``cam_center`` (Sec. 3.1)."""
    v = means - cam_center[None, :]
    dirs = v / torch.linalg.norm(v, dim=-1, keepdim=True)
    Y = basis(dirs, degree)                       # [n, nb]
    nb = (degree + 1) ** 2
    raw = (Y[:, :, None] * sh[:, :nb, :]).sum(1) + 0.5
    return torch.clamp(raw, min=0.0)
