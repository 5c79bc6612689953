"""Per-pixel ray evaluation in float64 (paper Sec. 3.2 and Sec. 3.3).

A pixel ray at window coordinates (x_s, y_s) is the intersection of the
screen planes pi_x = (1, 0, 0, -x_s) and pi_y = (0, 1, 0, -y_s). Planes map
to normalised splat space by the transpose of T' (Eq. ray-mapping), giving
pi_x^s = (a^1 : a^2 : a^3 : a^0) and pi_y^s = (b^1 : b^2 : b^3 : b^0), the
constant term last. The line's Pluecker coordinates are

  d = (p^23, p^31, p^12)   (direction)
  m = (p^01, p^02, p^03)   (moment),   p^ij = a^i b^j - a^j b^i

and rho^2 = |m|^2 / |d|^2 (Eq. rho-pluecker); |d| = 0 means the ray misses.
The point of maximum density on the ray is (d x m) / |d|^2 in splat space;
its view-space position is M T applied to that point (Sec. 3.3), and the
depth used for ordering is its z.
"""
from __future__ import annotations

import torch

F64 = torch.float64


def pixel_planes(xs, ys):
    """Screen planes (1,0,0,-x_s) and (0,1,0,-y_s) for window coordinates."""
    zeros = torch.zeros_like(xs)
    ones = torch.ones_like(xs)
    pi_x = torch.stack([ones, zeros, zeros, -xs], dim=-1)
    pi_y = torch.stack([zeros, ones, zeros, -ys], dim=-1)
    return pi_x, pi_y


def to_splat_space(Tp, pi):
    """(T')^T pi for every (pixel, Gaussian): Tp [g,4,4], pi [p,4] ->
    [p,g,4] with components ordered (coef of x, y, z, coef of w)."""
    return torch.einsum('grc,pr->pgc', Tp, pi)


def pluecker(a, b):
    """Dual-Pluecker construction of Sec. 3.2 from the two splat-space
    planes, components 0..2 = (a^1, a^2, a^3) and component 3 = a^0."""
    a1, a2, a3, a0 = a.unbind(-1)
    b1, b2, b3, b0 = b.unbind(-1)

    def p(ai, aj, bi, bj):
        return ai * bj - aj * bi

    d = torch.stack([p(a2, a3, b2, b3), p(a3, a1, b3, b1), p(a1, a2, b1, b2)], dim=-1)
    m = torch.stack([p(a0, a1, b0, b1), p(a0, a2, b0, b2), p(a0, a3, b0, b3)], dim=-1)
    return d, m


def rho2_and_depth(d, m, MT):
    """rho^2 = |m|^2/|d|^2 (inf where |d| = 0) and the view-space depth of
    the maximum-density point, z = (M T [ (d x m)/|d|^2 ; 1 ])_z."""
    dd = (d * d).sum(-1)
    mm = (m * m).sum(-1)
    hit = dd > 0
    safe = torch.where(hit, dd, torch.ones_like(dd))
    rho2 = torch.where(hit, mm / safe, torch.full_like(dd, float('inf')))
    x = torch.linalg.cross(d, m, dim=-1) / safe[..., None]        # [p,g,3]
    row = MT[:, 2, :]                                              # [g,4]
    z = (x * row[None, :, :3]).sum(-1) + row[None, :, 3]
    return rho2, z, hit
