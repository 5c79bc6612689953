"""Pins of the near-tie checker in tests/parity.py, on hand-made fragment
records of one pixel (CPU only). The checker must accept a GPU colour
that follows a branch float64 also admits, and reject one that follows a
wrong core order, leaves out a clearly eligible nearer fragment, or
blends a tail fragment that lies clearly outside the inclusion boundary."""
import numpy as np
import pytest
import torch

import oracle
from tests import parity
from tests import oracle_helpers as H

ST = H.settings(K=2, bg=(0.1, 0.2, 0.3))


def rec(frags):
    """frags: list of (gid, rho2, rho_c, raw alpha, depth, rgb)."""
    out = dict(gid=np.array([f[0] for f in frags]), rho2=np.array([f[1] for f in frags]),
               rho_c=np.array([f[2] for f in frags]), raw=np.array([f[3] for f in frags]),
               depth=np.array([f[4] for f in frags]),
               colour=np.array([f[5] for f in frags], np.float64))
    out['frag'] = out['rho2'] <= out['rho_c']
    return out


def composite(r, core, tail):
    a = np.minimum(ST.alpha_max, r['raw'])
    pos = {int(g): i for i, g in enumerate(r['gid'])}
    ci = [pos[g] for g in core]
    ti = [pos[g] for g in tail]
    return oracle.blend.composite_pixel([torch.tensor(a[i]) for i in ci],
                                        [torch.tensor(r['colour'][i]) for i in ci],
                                        [torch.tensor(a[i]) for i in ti],
                                        [torch.tensor(r['colour'][i]) for i in ti],
                                        ST.bg).numpy()


R = (1.0, 0.2, 0.1)
G = (0.1, 0.9, 0.2)
B = (0.2, 0.1, 0.8)
W = (0.7, 0.7, 0.7)


def test_accepts_the_plain_branch():
    r = rec([(3, 1.0, 9.0, 0.6, 2.0, R), (5, 2.0, 9.0, 0.5, 3.0, G), (8, 3.0, 9.0, 0.4, 4.0, B)])
    rgb = composite(r, [3, 5], [8])
    assert parity.recompute_with_branch(r, [3, 5], ST, rgb) < 1e-12


def test_rejects_swapped_core_order():
    r = rec([(3, 1.0, 9.0, 0.6, 2.0, R), (5, 2.0, 9.0, 0.5, 3.0, G), (8, 3.0, 9.0, 0.4, 4.0, B)])
    rgb = composite(r, [5, 3], [8])
    assert parity.recompute_with_branch(r, [5, 3], ST, rgb) is None


def test_accepts_swapped_core_order_at_a_depth_tie():
    r = rec([(3, 1.0, 9.0, 0.6, 3.0, R), (5, 2.0, 9.0, 0.5, 3.0 * (1 + 2e-6), G),
             (8, 3.0, 9.0, 0.4, 4.0, B)])
    rgb = composite(r, [5, 3], [8])
    assert abs(rgb - composite(r, [3, 5], [8])).max() > 1e-2     # the branches differ
    assert parity.recompute_with_branch(r, [5, 3], ST, rgb) < 1e-12


def test_rejects_a_core_that_misses_a_nearer_eligible_fragment():
    r = rec([(3, 1.0, 9.0, 0.6, 2.0, R), (5, 2.0, 9.0, 0.5, 3.0, G), (8, 3.0, 9.0, 0.4, 4.0, B)])
    rgb = composite(r, [5, 8], [3])
    assert parity.recompute_with_branch(r, [5, 8], ST, rgb) is None


def test_rejects_a_short_core_that_leaves_out_an_eligible_fragment():
    r = rec([(3, 1.0, 9.0, 0.6, 2.0, R), (5, 2.0, 9.0, 0.5, 3.0, G)])
    rgb = composite(r, [3], [5])
    assert parity.recompute_with_branch(r, [3], ST, rgb) is None


def test_rejects_an_ineligible_core_member():
    # alpha 0.01 < tau_K = 0.05: never a core member
    r = rec([(3, 1.0, 9.0, 0.01, 2.0, R), (5, 2.0, 9.0, 0.5, 3.0, G)])
    rgb = composite(r, [3, 5], [])
    assert parity.recompute_with_branch(r, [3, 5], ST, rgb) is None


def test_accepts_an_eligibility_tie():
    # alpha within 1e-4 of tau_K: core or tail are both admissible
    a = ST.tau_core * (1 - 5e-5)
    r = rec([(3, 1.0, 9.0, 0.6, 2.0, R), (5, 2.0, 9.0, a, 3.0, G), (8, 3.0, 9.0, 0.4, 4.0, B)])
    rgb = composite(r, [3, 5], [8])
    assert parity.recompute_with_branch(r, [3, 5], ST, rgb) < 1e-12


def test_tail_with_a_fragment_clearly_outside_the_cutoff_is_rejected():
    r = rec([(3, 1.0, 9.0, 0.6, 2.0, R), (5, 2.0, 9.0, 0.5, 3.0, G), (8, 3.0, 9.0, 0.4, 4.0, B),
             (9, 9.0 * 1.005, 9.0, 0.3, 5.0, W)])
    assert not r['frag'][3]
    rgb = composite(r, [3, 5], [8, 9])
    err = parity.recompute_with_branch(r, [3, 5], ST, rgb)
    assert err is not None and err > 1e-4


def test_tail_with_a_fragment_at_the_cutoff_is_accepted():
    r = rec([(3, 1.0, 9.0, 0.6, 2.0, R), (5, 2.0, 9.0, 0.5, 3.0, G), (8, 3.0, 9.0, 0.4, 4.0, B),
             (9, 9.0 * (1 + 3e-5), 9.0, 0.3, 5.0, W)])
    assert not r['frag'][3]
    rgb = composite(r, [3, 5], [8, 9])
    assert parity.recompute_with_branch(r, [3, 5], ST, rgb) < 1e-12
    # and so is the branch that leaves it out
    rgb2 = composite(r, [3, 5], [8])
    assert parity.recompute_with_branch(r, [3, 5], ST, rgb2) < 1e-12


def test_dropped_tail_fragment_is_rejected():
    r = rec([(3, 1.0, 9.0, 0.6, 2.0, R), (5, 2.0, 9.0, 0.5, 3.0, G), (8, 3.0, 9.0, 0.4, 4.0, B),
             (9, 4.0, 9.0, 0.3, 5.0, W)])
    rgb = composite(r, [3, 5], [8])
    err = parity.recompute_with_branch(r, [3, 5], ST, rgb)
    assert err is not None and err > 1e-4


def _info_of(pixels):
    """info['frags'] of a 1 x len(pixels) image from per-pixel records."""
    keys = ('gid', 'rho2', 'rho_c', 'raw', 'depth', 'colour', 'frag')
    out = {k: np.concatenate([p[k] for p in pixels]) for k in keys}
    out['pix'] = np.concatenate([np.full(p['gid'].size, i) for i, p in enumerate(pixels)])
    out['ptr'] = np.searchsorted(out['pix'], np.arange(len(pixels) + 1))
    return dict(frags=out)


def test_check_image_counts_resolved_and_unresolved_pixels():
    good = rec([(3, 1.0, 9.0, 0.6, 2.0, R), (5, 2.0, 9.0, 0.5, 2.0 * (1 + 1e-6), G)])
    bad = rec([(3, 1.0, 9.0, 0.6, 2.0, R), (5, 2.0, 9.0, 0.5, 3.0, G)])
    info = _info_of([good, bad])
    ref = np.stack([composite(good, [3, 5], []), composite(bad, [3, 5], [])], 1)[:, None, :]
    gpu = np.stack([composite(good, [5, 3], []), composite(bad, [5, 3], [])], 1)[:, None, :]
    core = np.array([[5, 5], [3, 3]])[:, None, :]
    with pytest.raises(AssertionError):
        parity.check_image(gpu.astype(np.float32), core, ref, info, ST)
    stats = parity.check_image(gpu.astype(np.float32), core, ref, info, ST, max_unresolved=1)
    assert stats['n_bad'] == 2 and stats['resolved'] == 1 and len(stats['unresolved']) == 1


def test_ambiguous_pixels_marks_each_kind_of_tie():
    plain = rec([(3, 1.0, 9.0, 0.6, 2.0, R), (5, 2.0, 9.0, 0.5, 3.0, G)])
    ztie = rec([(3, 1.0, 9.0, 0.6, 2.0, R), (5, 2.0, 9.0, 0.5, 2.0 * (1 + 1e-6), G)])
    cut = rec([(3, 9.0 * (1 - 1e-5), 9.0, 0.6, 2.0, R)])
    elig = rec([(3, 1.0, 9.0, ST.tau_core * (1 + 1e-5), 2.0, R)])
    clamp = rec([(3, 1.0, 9.0, ST.alpha_max * (1 + 1e-5), 2.0, R)])
    deep = rec([(3, 1.0, 9.0, 0.6, 2.0, R), (5, 2.0, 9.0, 0.5, 3.0, G), (7, 2.0, 9.0, 0.5, 4.0, B),
                (8, 2.0, 9.0, 0.5, 4.0 * (1 + 1e-6), W)])   # tie behind the core boundary
    info = _info_of([plain, ztie, cut, elig, clamp, deep])
    amb = parity.ambiguous_pixels(info, 1, 6, ST)[0]
    assert amb.tolist() == [False, True, True, True, True, False]


# ---------------------------------------------------------------------------
# Sorted blending (alpha blending in mean-depth order with an early stop)
# ---------------------------------------------------------------------------

def sorted_settings(tau_T):
    return H.settings(K=2, bg=(0.1, 0.2, 0.3), sorted_blend=True, tau_T=tau_T)


def blend_in_order(r, gids, st):
    """Float64 Eq. alpha_blending over the given Gaussians, then the
    background."""
    a = np.minimum(st.alpha_max, r['raw'])
    pos = {int(g): i for i, g in enumerate(r['gid'])}
    T, C = 1.0, np.zeros(3)
    for g in gids:
        i = pos[g]
        C = C + a[i] * T * r['colour'][i]
        T *= 1.0 - a[i]
    return C + T * np.asarray(st.bg)


# mean depths that order the Gaussians 8, 3, 5, 9 (index ties broken by index)
ORDER_KEY = np.zeros(16, np.float32)
ORDER_KEY[[8, 3, 5, 9]] = [1.0, 2.0, 3.0, 4.0]
FRAGS = [(3, 1.0, 9.0, 0.6, 2.0, R), (5, 2.0, 9.0, 0.5, 3.0, G), (8, 3.0, 9.0, 0.4, 4.0, B),
         (9, 1.5, 9.0, 0.9, 1.0, W)]


def test_sorted_accepts_the_plain_branch_and_rejects_wrong_ones():
    r = rec(FRAGS)
    st = sorted_settings(1e-4)
    # transmittance stays above 1e-4: all four blended in the order 8, 3, 5, 9
    rgb = blend_in_order(r, [8, 3, 5, 9], st)
    assert parity.sorted_branch_error(r, ORDER_KEY, st, 4, -1, rgb) < 1e-12
    # index order instead of depth order
    bad = blend_in_order(r, [3, 5, 8, 9], st)
    assert parity.sorted_branch_error(r, ORDER_KEY, st, 4, -1, bad) > 1e-3
    # a stop the transmittance does not call for
    assert parity.sorted_branch_error(r, ORDER_KEY, st, 2, 5,
                                      blend_in_order(r, [8, 3], st)) is None
    # a count that does not match the stop position
    assert parity.sorted_branch_error(r, ORDER_KEY, st, 3, -1, rgb) is None


def test_sorted_early_stop_branch():
    r = rec(FRAGS)
    # after 8 and 3: T = 0.6 * 0.4 = 0.24; 5 would take it to 0.12
    st = sorted_settings(0.15)
    rgb = blend_in_order(r, [8, 3], st)
    assert parity.sorted_branch_error(r, ORDER_KEY, st, 2, 5, rgb) < 1e-12
    # blending past the stop is wrong
    assert parity.sorted_branch_error(r, ORDER_KEY, st, 3, 9,
                                      blend_in_order(r, [8, 3, 5], st)) is None
    # stopping a fragment early is wrong too
    assert parity.sorted_branch_error(r, ORDER_KEY, st, 1, 3,
                                      blend_in_order(r, [8], st)) is None


def test_sorted_accepts_either_side_of_a_threshold_tie():
    r = rec(FRAGS)
    # tau_T a hair above T after 8, 3, 5 (0.12): stopping at 5 or not are
    # both admissible
    st = sorted_settings(0.12 * (1 + 3e-5))
    stop = blend_in_order(r, [8, 3], st)
    go_on = blend_in_order(r, [8, 3, 5], st)
    assert parity.sorted_branch_error(r, ORDER_KEY, st, 2, 5, stop) < 1e-12
    assert parity.sorted_branch_error(r, ORDER_KEY, st, 3, 9, go_on) < 1e-12
    # but not far from the threshold
    st_far = sorted_settings(0.13)
    assert parity.sorted_branch_error(r, ORDER_KEY, st_far, 3, 9,
                                      blend_in_order(r, [8, 3, 5], st_far)) is None


def test_sorted_inclusion_tie_either_way_but_not_a_clear_miss():
    # Gaussian 5 sits at the inclusion boundary; Gaussian 9 clearly outside
    frags = [(3, 1.0, 9.0, 0.6, 2.0, R), (5, 9.0 * (1 + 5e-5), 9.0, 0.5, 3.0, G),
             (8, 3.0, 9.0, 0.4, 4.0, B), (9, 9.5, 9.0, 0.9, 1.0, W)]
    r = rec(frags)
    st = sorted_settings(1e-4)
    assert parity.sorted_branch_error(r, ORDER_KEY, st, 3, -1,
                                      blend_in_order(r, [8, 3, 5], st)) < 1e-12
    assert parity.sorted_branch_error(r, ORDER_KEY, st, 2, -1,
                                      blend_in_order(r, [8, 3], st)) < 1e-12
    e = parity.sorted_branch_error(r, ORDER_KEY, st, 3, -1, blend_in_order(r, [8, 3, 9], st))
    assert e is None or e > 1e-3
