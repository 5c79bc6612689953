"""Autotuner: picks the tile shape, the forward LDS batch depth and the tile
order for a workload by timing a few forward+backward steps of each
candidate on the device (HIP events), and caches the choice as JSON.

Environment: HTGS_TUNE = search (default) | cache (use the cache, search on
a miss) | off (keep the given settings); HTGS_TUNE_CACHE = path of the JSON
cache (default ~/.cache/htgs_tune.json). The cache key is the device name,
log2 buckets of the Gaussian count and of the total pixel count, the number
of views, K and the SH degree.
"""
from __future__ import annotations

import dataclasses
import json
import math
import os

import torch

from . import htgs

CANDIDATES = (
    # (tile width, tile height, lds_batch multiplier, cost order, tile culling,
    #  persistent tile queue)
    (8, 8, 1, False, False, False), (8, 8, 2, False, False, False),
    (8, 8, 1, True, False, False), (8, 8, 2, True, False, False),
    (16, 8, 1, False, False, False), (16, 16, 1, False, False, False),
    (16, 16, 1, True, False, False), (32, 8, 1, False, False, False),
    (8, 8, 1, False, True, False), (8, 8, 1, True, True, False),
    (16, 8, 1, False, True, False), (16, 8, 1, True, True, False),
    (16, 16, 1, False, True, False), (16, 16, 1, True, True, False),
    (32, 8, 1, False, True, False), (32, 8, 1, True, True, False),
    (8, 8, 1, False, True, True), (8, 8, 1, True, True, True),
    (16, 8, 1, False, True, True), (16, 8, 1, True, True, True),
    (16, 16, 1, False, True, True), (16, 16, 1, True, True, True),
)


def _cache_path():
    return os.environ.get("HTGS_TUNE_CACHE", os.path.expanduser("~/.cache/htgs_tune.json"))


def _key(n, cams, st, sh_degree):
    px = sum(c.width * c.height for c in cams)
    dev = torch.cuda.get_device_name(0) if torch.cuda.is_available() else "cpu"
    return (f"v4|{dev}|n{int(math.log2(max(n, 1)))}|px{int(math.log2(max(px, 1)))}|v{len(cams)}"
            f"|K{st.K}|sh{sh_degree}")


def candidate_name(cand):
    return (f"tile{cand[0]}x{cand[1]}_batch{cand[2]}x_{'cost' if cand[3] else 'xcd'}"
            f"{'_cull' if cand[4] else ''}{'_queue' if cand[5] else ''}")


def by_name(name):
    """The candidate called ``name`` (as in the tuning reports)."""
    for cand in CANDIDATES:
        if candidate_name(cand) == name:
            return cand
    raise KeyError(f"unknown schedule {name!r}; one of "
                   + ", ".join(candidate_name(c) for c in CANDIDATES))


def apply(st, cand):
    tw, th, mult, order, cull, persist = cand
    return dataclasses.replace(st, tile_w=tw, tile_h=th,
                               lds_batch=(tw * th * mult) if mult > 1 else 0,
                               cost_order=bool(order), tile_cull=bool(cull),
                               persistent=bool(persist))


def _time_candidate(params, sh_degree, cams, st, steps):
    dev = params[0].device
    n_inst = htgs.count_instances(params, sh_degree, cams, st)
    ws = htgs.alloc_workspace(params[0].shape[0], cams, st, n_inst, dev)
    state = torch.empty(htgs.state_bytes(cams, st) // 4, dtype=torch.float32, device=dev)
    imgs = [torch.empty((3, c.height, c.width), dtype=torch.float32, device=dev) for c in cams]
    gimgs = [torch.full_like(im, 1.0 / im.numel()) for im in imgs]
    grads = [torch.zeros_like(p) for p in params]

    def step():
        fr = htgs.forward(params, sh_degree, cams, st, ws=ws, state=state, images=imgs)
        htgs.backward(params, fr, gimgs, grads=grads)

    step()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        step()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def tune(params, sh_degree, cams, st, steps=3, verbose=False, cull_choices=None):
    """Returns (settings, report) for this workload. cull_choices restricts
    the tile-culling setting of the candidates (None: both)."""
    mode = os.environ.get("HTGS_TUNE", "search")
    if mode == "off":
        return st, {"mode": "off"}
    key = _key(params[0].shape[0], cams, st, sh_degree) + (
        "" if cull_choices is None else f"|cull{sorted(cull_choices)}")
    path = _cache_path()
    cache = {}
    if os.path.exists(path):
        try:
            cache = json.load(open(path))
        except (OSError, ValueError):
            cache = {}
    if mode == "cache" and key in cache:
        return apply(st, tuple(cache[key]["choice"])), {"mode": "cache", **cache[key]}
    times = {}
    named = {}
    for cand in CANDIDATES:
        if cand[0] * cand[1] > 128 and st.K > 16:
            continue
        if cull_choices is not None and cand[4] not in cull_choices:
            continue
        ms = _time_candidate(params, sh_degree, cams, apply(st, cand), steps)
        name = candidate_name(cand)
        times[name] = ms
        named[name] = cand
        if verbose:
            print(f"autotune {name}: {ms:.3f} ms", flush=True)
    # the few fastest are timed again over more steps, so that run-to-run
    # noise in the short first pass does not decide between near-equals
    finalists = sorted(times, key=times.get)[:3]
    refined = {name: _time_candidate(params, sh_degree, cams, apply(st, named[name]), 3 * steps)
               for name in finalists}
    best = min(refined, key=refined.get)
    choice = named[best]
    entry = {"choice": list(choice), "best": best, "ms": times, "refined_ms": refined}
    cache[key] = entry
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        json.dump(cache, open(path, "w"), indent=1)
    except OSError:
        pass
    return apply(st, choice), {"mode": "search", **entry}
