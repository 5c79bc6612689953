"""GPU-vs-oracle comparison helpers (test code).

Tile lists: bit-exact, except instances of Gaussians whose float64 box edge
lies within 1e-9 of a pixel-centre boundary (a round-off tie, reported).

Images: max-abs 1e-4 per pixel. A pixel above that is accepted only if it is
a near-tie pixel and the GPU's branch is admissible: its core (exported in
the forward state) consists of fragments whose alpha is at least tau_K
within 1e-4, in depth order within 1e-5 relative, with no clearly eligible
fragment left out in front of the last core member; and the float64
composite recomputed with the GPU's core and some choice of the fragments
that sit within 1e-4 (relative) of the inclusion boundary rho^2 = rho_c
matches the GPU colour within 1e-4.
"""
from __future__ import annotations

import itertools

import numpy as np
import torch

import oracle

TOL_IMG = 1e-4
DELTA_RHO = 1e-4
DELTA_Z = 1e-5
DELTA_A = 1e-4


def compare_bins(gpu_keys, gpu_vals, gpu_rects, ref, margin_tol=1e-9):
    amb = np.nonzero(ref['margin'] < margin_tol)[0]
    n = ref['tile_rect'].shape[0]
    gr = gpu_rects.astype(np.int64)
    g_empty = gr[:, 0] > gr[:, 2]
    r_empty = ~ref['nonempty']
    mask = np.ones(n, bool)
    mask[amb] = False
    assert (g_empty[mask] == r_empty[mask]).all(), "empty-rect mismatch"
    both = mask & ~r_empty
    assert (gr[both] == ref['tile_rect'][both]).all(), "tile rect mismatch"
    k, v = gpu_keys.astype(np.int64), gpu_vals.astype(np.int64)
    rk, rv = ref['keys'], ref['values']
    if amb.size:
        keep_g = ~np.isin(v, amb)
        keep_r = ~np.isin(rv, amb)
        k, v, rk, rv = k[keep_g], v[keep_g], rk[keep_r], rv[keep_r]
    assert k.shape == rk.shape, (k.shape, rk.shape)
    assert (k == rk).all() and (v == rv).all(), "sorted lists differ"
    return int(amb.size)


def _pixel_records(frags, p):
    a, b = frags['ptr'][p], frags['ptr'][p + 1]
    return {key: frags[key][a:b] for key in ('gid', 'rho2', 'rho_c', 'raw', 'depth', 'colour',
                                             'frag')}


def _admissible(rec, core, st):
    K = int(st.K)
    gid = rec['gid']
    alpha = np.minimum(st.alpha_max, rec['raw'])
    clear_in = rec['rho2'] < rec['rho_c'] * (1 - DELTA_RHO)
    amb_in = np.abs(rec['rho2'] - rec['rho_c']) <= DELTA_RHO * rec['rho_c']
    pos = {int(g): i for i, g in enumerate(gid)}
    idx = []
    for c in core:
        if c not in pos:
            return None
        i = pos[c]
        if not (clear_in[i] or amb_in[i]):
            return None
        if alpha[i] < st.tau_core * (1 - DELTA_A):
            return None
        idx.append(i)
    z = rec['depth']
    for a_, b_ in zip(idx, idx[1:]):
        if z[b_] < z[a_] - DELTA_Z * abs(z[a_]):
            return None
    elig = clear_in & (alpha >= st.tau_core * (1 + DELTA_A))
    missing = [i for i in np.nonzero(elig)[0] if int(gid[i]) not in set(core)]
    if missing:
        if len(core) < K:
            return None
        zl = z[idx[-1]]
        if any(z[i] < zl - DELTA_Z * abs(zl) for i in missing):
            return None
    return idx, clear_in, amb_in, alpha


def recompute_with_branch(rec, core, st, gpu_rgb):
    """Smallest max-abs error over admissible branch choices (None if the
    GPU core is inadmissible or too many inclusion ties). Without the tail
    (st.no_tail) only the core is blended."""
    adm = _admissible(rec, core, st)
    if adm is None:
        return None
    idx, clear_in, amb_in, alpha = adm
    core_set = set(idx)
    amb_free = [i for i in np.nonzero(amb_in)[0] if i not in core_set]
    if getattr(st, 'no_tail', False):
        amb_free = []
    if len(amb_free) > 6:
        return None
    base_tail = [i for i in np.nonzero(clear_in & ~amb_in)[0] if i not in core_set]
    if getattr(st, 'no_tail', False):
        base_tail = []
    col = rec['colour']
    best = np.inf
    for r in range(len(amb_free) + 1):
        for sub in itertools.combinations(amb_free, r):
            tail = base_tail + list(sub)
            C = oracle.blend.composite_pixel(
                [torch.tensor(alpha[i]) for i in idx], [torch.tensor(col[i]) for i in idx],
                [torch.tensor(alpha[i]) for i in tail], [torch.tensor(col[i]) for i in tail],
                st.bg).numpy()
            best = min(best, float(np.abs(C - gpu_rgb).max()))
    return best


def check_image(gpu_img, gpu_core, ref_img, info, st, tol=TOL_IMG, max_unresolved=0):
    """gpu_img [3,H,W], gpu_core [K,H,W] int, ref_img [3,H,W] float64."""
    H, W = ref_img.shape[1:]
    err = np.abs(gpu_img.astype(np.float64) - ref_img).max(0)
    bad = np.argwhere(err > tol)
    resolved, unresolved = 0, []
    for (y, x) in bad:
        p = y * W + x
        rec = _pixel_records(info['frags'], p)
        core = [int(c) for c in gpu_core[:, y, x] if c >= 0]
        e = recompute_with_branch(rec, core, st, gpu_img[:, y, x].astype(np.float64))
        if e is not None and e <= tol:
            resolved += 1
        else:
            unresolved.append((int(y), int(x), float(err[y, x]), e))
    clean = err.copy()
    for (y, x) in bad:
        clean[y, x] = 0.0
    stats = dict(max_err=float(err.max()), max_err_clean=float(clean.max()), n_bad=int(len(bad)),
                 resolved=resolved, unresolved=unresolved)
    assert len(unresolved) <= max_unresolved, stats
    return stats


def ambiguous_pixels(info, H, W, st):
    """[H, W] bool: pixels holding a near-tie of the kind the image protocol
    arbitrates (a fragment within DELTA_RHO of rho^2 = rho_c, an alpha
    within DELTA_A of tau_K or of the clamp, or two eligible fragments
    among the front K + 1 whose depths lie within DELTA_Z). At such a pixel
    float32 may take either branch, and the gradient differs between the
    branches, so gradient windows leave these pixels out of the loss."""
    fr = info['frags']
    out = np.zeros(H * W, bool)
    if fr['pix'].size == 0:
        return out.reshape(H, W)
    rho2, rc, raw, z = fr['rho2'], fr['rho_c'], fr['raw'], fr['depth']
    alpha = np.minimum(st.alpha_max, raw)
    frag = fr['frag'].astype(bool)
    near = np.abs(rho2 - rc) <= DELTA_RHO * rc
    near |= frag & (np.abs(alpha - st.tau_core) <= DELTA_A * st.tau_core)
    near |= frag & (np.abs(raw - st.alpha_max) <= DELTA_A * st.alpha_max)
    np.logical_or.at(out, fr['pix'][near], True)
    K = int(st.K)
    elig = frag & (alpha >= st.tau_core)
    pix_e, z_e = fr['pix'][elig], z[elig]
    order = np.lexsort((z_e, pix_e))
    pix_e, z_e = pix_e[order], z_e[order]
    if pix_e.size > 1 and K > 0:
        start = np.searchsorted(pix_e, pix_e, side='left')
        rank = np.arange(pix_e.size) - start
        same = pix_e[1:] == pix_e[:-1]
        close = np.abs(z_e[1:] - z_e[:-1]) <= DELTA_Z * np.abs(z_e[:-1])
        hit = same & close & (rank[:-1] < K)
        np.logical_or.at(out, pix_e[1:][hit], True)
    return out.reshape(H, W)


def grad_errors(got, ref):
    """Per-tensor (|g - g_ref| / |g_ref|, max |g - g_ref| / max |g_ref|)."""
    out = []
    for a, b in zip(got, ref):
        a = np.asarray(a, np.float64)
        b = np.asarray(b, np.float64)
        den = np.linalg.norm(b)
        rel = np.linalg.norm(a - b) / max(den, 1e-30)
        elem = np.abs(a - b).max() / max(np.abs(b).max(), 1e-30) if b.size else 0.0
        out.append((float(den), float(rel), float(elem)))
    return out


DELTA_T = 1e-4


def sorted_branch_error(rec, order_key, st, nb, stop_gid, gpu_rgb):
    """Sorted blending at one pixel: the smallest max-abs error of the float64
    composite over the branches the GPU's decisions admit, or None if none
    does. The fragments run front to back by (order_key[gid], gid); those
    within DELTA_RHO of rho^2 = rho_c may count as fragments or not. A branch
    is admissible if the GPU blended exactly the first nb fragments before
    its stop fragment (all of them without a stop), every blended step kept
    the float64 transmittance at tau_T (1 - DELTA_T) or above, and the stop
    fragment takes it below tau_T (1 + DELTA_T)."""
    gid = rec['gid'].astype(np.int64)
    clear_in = rec['rho2'] < rec['rho_c'] * (1 - DELTA_RHO)
    amb_in = np.abs(rec['rho2'] - rec['rho_c']) <= DELTA_RHO * rec['rho_c']
    alpha = np.minimum(st.alpha_max, rec['raw'])
    col = rec['colour']
    order = np.lexsort((gid, order_key[gid]))
    amb = [i for i in order if amb_in[i]]
    if len(amb) > 6:
        return None
    tau = float(st.tau_T)
    bg = np.asarray(st.bg, np.float64)
    best = None
    for r in range(len(amb) + 1):
        for sub in itertools.combinations(amb, r):
            chosen = set(sub)
            L = [i for i in order if (clear_in[i] and not amb_in[i]) or i in chosen]
            if stop_gid >= 0:
                k = [j for j, i in enumerate(L) if gid[i] == stop_gid]
                if not k:
                    continue
                k = k[0]
            else:
                k = len(L)
            if k != nb:
                continue
            T, C, ok = 1.0, np.zeros(3), True
            for i in L[:k]:
                tn = T * (1.0 - alpha[i])
                if tn < tau * (1 - DELTA_T):
                    ok = False
                    break
                C = C + alpha[i] * T * col[i]
                T = tn
            if not ok:
                continue
            if stop_gid >= 0 and not (T * (1.0 - alpha[L[k]]) < tau * (1 + DELTA_T)):
                continue
            e = float(np.abs(C + T * bg - gpu_rgb).max())
            best = e if best is None else min(best, e)
    return best


def check_sorted_image(gpu_img, gpu_nb, gpu_stop, ref_img, info, order_key, st, tol=TOL_IMG,
                       max_unresolved=0):
    """Sorted blending: gpu_img [3,H,W], gpu_nb / gpu_stop [H,W] (blended
    fragment counts and stop Gaussians from the forward state), ref_img
    [3,H,W] float64; order_key[g]: the float32 mean depth the lists are
    sorted by. Pixels above tol must be near-ties whose GPU branch is
    admissible and matches its float64 recomputation within tol. Also
    reports how many pixels' (nb, stop) differ from the oracle's."""
    H, W = ref_img.shape[1:]
    err = np.abs(gpu_img.astype(np.float64) - ref_img).max(0)
    ref_core = info['core'].numpy()
    same_branch = (ref_core[..., 0] == gpu_nb) & (ref_core[..., 1] == gpu_stop)
    bad = np.argwhere((err > tol) | ~same_branch)
    resolved, unresolved = 0, []
    for (y, x) in bad:
        rec = _pixel_records(info['frags'], y * W + x)
        e = sorted_branch_error(rec, order_key, st, int(gpu_nb[y, x]), int(gpu_stop[y, x]),
                                gpu_img[:, y, x].astype(np.float64))
        if e is not None and e <= tol:
            resolved += 1
        else:
            unresolved.append((int(y), int(x), float(err[y, x]), e))
    clean = err.copy()
    for (y, x) in bad:
        clean[y, x] = 0.0
    stats = dict(max_err=float(err.max()), max_err_clean=float(clean.max()), n_bad=int(len(bad)),
                 branch_differs=int((~same_branch).sum()), resolved=resolved,
                 unresolved=unresolved[:10])
    assert len(unresolved) <= max_unresolved, stats
    return stats


def sorted_ambiguous_pixels(info, H, W, st, order_key):
    """[H, W] bool for sorted blending: pixels holding a near-tie that
    float32 may decide either way (a fragment within DELTA_RHO of rho^2 =
    rho_c, an alpha within DELTA_A of the clamp, or a step of the float64
    front-to-back transmittance within DELTA_T of tau_T); gradient windows
    leave them out of the loss."""
    fr = info['frags']
    out = np.zeros(H * W, bool)
    if fr['pix'].size == 0:
        return out.reshape(H, W)
    tau = float(st.tau_T)
    for p in np.unique(fr['pix']):
        rec = _pixel_records(fr, int(p))
        rho2, rc = rec['rho2'], rec['rho_c']
        if np.any(np.abs(rho2 - rc) <= DELTA_RHO * rc):
            out[p] = True
            continue
        frag = rec['frag'].astype(bool)
        if np.any(frag & (np.abs(rec['raw'] - st.alpha_max) <= DELTA_A * st.alpha_max)):
            out[p] = True
            continue
        gid = rec['gid'].astype(np.int64)
        order = [i for i in np.lexsort((gid, order_key[gid])) if frag[i]]
        T = 1.0
        for i in order:
            T *= 1.0 - min(st.alpha_max, rec['raw'][i])
            if abs(T - tau) <= DELTA_T * tau:
                out[p] = True
            if T < tau:
                break
    return out.reshape(H, W)
