"""Hybrid-transparency composite (paper Sec. 3.3, Eq. pixel_color_computation
and its helper equation).

The core is the K front-most fragments whose alpha is at least tau_K (the
second threshold of Sec. 4.2), alpha-blended in exact depth order; every other
fragment forms the tail, blended without order:

  C = sum_{i<=n} alpha_i T_i c_i + T_{n+1} ((1 - T_tail) c_tail + T_tail c_bg)
  T_i = prod_{j<i} (1 - alpha_j)
  c_tail = sum_tail alpha c / sum_tail alpha,  T_tail = prod_tail (1 - alpha)

Readings where the paper is silent: n is the number of actual core members
(n <= K) and T_{n+1} the transmittance after them; an empty tail contributes
T_{n+1} c_bg; equal depths are ordered by ascending Gaussian index.

Inference without the tail (Sec. 4.3, "Hybrid Transparency Ablations",
Table ablations): the tail term is left out, so the background lies
directly behind the core, C = sum_{i<=n} alpha_i T_i c_i + T_{n+1} c_bg.

Sorted blending (``sorted_alpha``, the paper's "w/o per-pixel HT"
configuration): no core and no tail; Eq. alpha_blending over each pixel's
fragments in the global front-to-back order of the Gaussians' mean depths,
with the 3DGS early stop at a transmittance threshold.
"""
from __future__ import annotations

import torch

F64 = torch.float64


def composite_pixel(core_alpha, core_colour, tail_alpha, tail_colour, bg):
    """One pixel, written out term by term. ``core_*`` are in depth order."""
    C = torch.zeros(3, dtype=F64)
    T = torch.ones((), dtype=F64)
    for a, c in zip(core_alpha, core_colour):
        C = C + a * T * c
        T = T * (1.0 - a)
    bg = torch.as_tensor(bg, dtype=F64)
    A = torch.zeros((), dtype=F64)
    S = torch.zeros(3, dtype=F64)
    P = torch.ones((), dtype=F64)
    for a, c in zip(tail_alpha, tail_colour):
        A = A + a
        S = S + a * c
        P = P * (1.0 - a)
    X = P * bg
    if float(A) > 0.0:
        X = X + (1.0 - P) * S / A
    return C + T * X


def hybrid(alpha, colour, depth, frag, K, tau_core, bg, tail=True):
    """Vectorised over pixels: alpha/depth/frag [P,G] (alpha = 0 off the
    fragments), colour [G,3]. Returns C [P,3] and per-pixel core indices
    (ordered, [P,min(K,G)], -1 past the n-th) for parity checks. With
    ``tail=False`` the tail term is dropped (inference without the tail)."""
    Pn, G = alpha.shape
    bg = torch.as_tensor(bg, dtype=F64)
    eligible = frag & (alpha >= tau_core)
    kk = min(int(K), G)
    n = torch.clamp(eligible.sum(1), max=kk)
    if kk > 0:
        key = torch.where(eligible, depth.detach(), torch.full_like(depth.detach(), float('inf')))
        order = torch.sort(key, dim=1, stable=True).indices[:, :kk]          # [P,kk]
        valid = torch.arange(kk)[None, :] < n[:, None]
        a_core = alpha.gather(1, order) * valid
        c_core = colour[order]                                             # [P,kk,3]
        one_minus = 1.0 - a_core
        T_incl = torch.cumprod(one_minus, dim=1)
        T_excl = torch.cat([torch.ones((Pn, 1), dtype=F64), T_incl[:, :-1]], dim=1)
        core_sum = ((a_core * T_excl)[:, :, None] * c_core).sum(1)
        T_n1 = T_incl[:, -1]
        core_mask = torch.zeros((Pn, G), dtype=torch.bool)
        core_mask.scatter_(1, order, valid)
        core_ids = torch.where(valid, order, torch.full_like(order, -1))
    else:
        core_sum = torch.zeros((Pn, 3), dtype=F64)
        T_n1 = torch.ones(Pn, dtype=F64)
        core_mask = torch.zeros((Pn, G), dtype=torch.bool)
        core_ids = torch.zeros((Pn, 0), dtype=torch.long)
    if not tail:
        C = core_sum + T_n1[:, None] * bg[None, :]
        return C, core_ids
    tail = frag & ~core_mask
    a_tail = torch.where(tail, alpha, torch.zeros_like(alpha))
    A = a_tail.sum(1)
    S = a_tail @ colour
    P = torch.prod(torch.where(tail, 1.0 - alpha, torch.ones_like(alpha)), dim=1)
    has_tail = A > 0
    A_safe = torch.where(has_tail, A, torch.ones_like(A))
    c_tail = S / A_safe[:, None]
    X = torch.where(has_tail[:, None], (1.0 - P)[:, None] * c_tail,
                    torch.zeros_like(c_tail)) + P[:, None] * bg[None, :]
    C = core_sum + T_n1[:, None] * X
    return C, core_ids


def sorted_alpha(alpha, colour, frag, order, tau_T, bg):
    """Alpha blending in one global order with an early stop (Sec. 4.3,
    "Perspectively Correct Splat Evaluation", Table splat_eval: the
    per-pixel evaluation of Sec. 3.2 combined with the approximately
    depth-ordered blending of 3DGS instead of hybrid transparency; Sec. 5,
    "Limitations and Future Work": plain alpha blending may stop once the
    transmittance falls below a preset threshold).

    ``order`` [G] lists the Gaussians front to back by the view depth of
    their means (the same order for every pixel; ties by ascending index,
    the caller's stable sort). Per pixel, Eq. alpha_blending runs over its
    fragments in that order; the first fragment that would bring the
    transmittance below tau_T is left out, and so is everything after it
    (the 3DGS rule). C = sum_blended alpha_i T_i c_i + T_end c_bg.

    alpha/frag [P,G] (alpha = 0 off the fragments), colour [G,3]. Returns C
    [P,3], the number of blended fragments per pixel and the index (into
    the G columns) of the fragment the stop left out, -1 if none."""
    Pn, G = alpha.shape
    bg = torch.as_tensor(bg, dtype=F64)
    a = alpha[:, order]
    f = frag[:, order]
    one_minus = 1.0 - a
    T_incl = torch.cumprod(one_minus, dim=1)
    T_excl = torch.cat([torch.ones((Pn, 1), dtype=F64), T_incl[:, :-1]], dim=1)
    stop_here = f & (T_incl.detach() < tau_T)
    # everything from the first stop on is left out
    stopped = torch.cumsum(stop_here.to(torch.int64), dim=1) > 0
    blended = f & ~stopped
    w = torch.where(blended, a * T_excl, torch.zeros_like(a))
    C = w @ colour[order]
    # transmittance after the last blended fragment
    T_end = torch.prod(torch.where(blended, one_minus, torch.ones_like(one_minus)), dim=1)
    C = C + T_end[:, None] * bg[None, :]
    first = torch.where(stop_here.any(1), stop_here.to(torch.int64).argmax(1),
                        torch.full((Pn,), -1, dtype=torch.int64))
    stop_col = torch.where(first >= 0, order[first.clamp(min=0)], first)
    return C, blended.sum(1), stop_col


def depth_order(mean_depth32):
    """Front-to-back order of Gaussians by the float32 view depth of their
    means, ties by ascending index (a stable sort)."""
    return torch.sort(torch.as_tensor(mean_depth32), stable=True).indices
