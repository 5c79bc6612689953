#!/usr/bin/env python3
"""Benchmark of the hot path on one MI355X, through the C ABI.

A step is one forward render + the L1-loss image gradient + the backward.
Default workload: 1M clustered Gaussians (SH degree 3), one 1920x1080
camera, K = 8; tile shape, forward LDS batch depth and tile order picked by
the autotuner. Inputs are resident in HBM before timing. Prints ONE JSON
line on stdout; progress goes to stderr.

    python bench.py [--steps K] [--warmup W] [--workload 1080p|720p|small|stress|multiview]

The default run also measures the batched multi-view step (3M Gaussians,
16 views of uneven resolution): 16 sequential single-view fwd+bwd calls of
the same kernels versus one replay of a hipGraph holding the batched
fwd+bwd; reported under "multiview" (skip with --no-multiview).
"""
from __future__ import annotations

import argparse
import dataclasses
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Peaks (MI355X spec sheet): HBM3E 8 TB/s; FP32 vector FMA without packed
# instructions: 256 CUs x 64 lanes x 2 flop x 2.4 GHz = 78.6 TFLOP/s.
HBM_PEAK_GBS = 8000.0
FP32_PEAK_TFLOPS = 256 * 64 * 2 * 2.4e9 / 1e12

# Algorithmic float32 flops of the rasterizer (FMA = 2): a candidate pair
# (tile pixel x tile instance) evaluates d, m, |d|^2, |m|^2 and the cutoff
# test; a fragment adds alpha and its tail (forward) or its adjoint
# (backward) work. Core insertion is not counted.
FLOPS_PAIR = 35
FLOPS_FRAG_FWD = 15
FLOPS_FRAG_BWD = 64


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def workload(name):
    from paper_2410_08129_amd import scenes
    if name == "1080p":
        sc, cams, st = scenes.workload_1080p()
        desc = "1M clustered Gaussians, SH3, 1920x1080, fov 50, K=8, fwd+bwd (L1 to smooth target)"
    elif name == "720p":
        sc, cams, st = scenes.workload_720p()
        desc = "1M clustered Gaussians, SH3, 1280x720, fov 50, K=8, fwd+bwd (L1 to smooth target)"
    elif name == "small":
        sc, cams, st = scenes.workload_small()
        desc = "4096 uniform Gaussians, SH0, 128x128, fov 60, K=4, fwd+bwd"
    elif name == "stress":
        sc, cams, st = scenes.workload_stress()
        desc = ("6M clustered Gaussians (10% zero-axis, 2% 1e-7-axis), SH3, 3840x2160, fov 70, "
                "K=16, fwd+bwd")
    elif name == "multiview":
        sc, cams, st = scenes.workload_multiview()
        desc = ("3M clustered Gaussians (128 clusters), SH3, 16 views of uneven resolution, "
                "fov 50, K=8, fwd+bwd")
    else:
        raise SystemExit(f"unknown workload {name}")
    return sc, cams, st, desc


def cpu_baseline(sc, cam, st, min_seconds=10.0, max_crops=64, size=64):
    """The FP64 oracle on a bounded sample: forward + autograd backward of
    seeded 64x64 crops (as many as fit in about min_seconds, at least 2);
    extrapolated to the full frame by pixel count."""
    import torch

    import oracle
    from paper_2410_08129_amd import scenes
    torch.set_num_threads(os.cpu_count() or 1)
    crops = scenes.random_crops(cam, max_crops, size, seed=5)
    target = scenes.smooth_target(cam.height, cam.width)
    t0 = time.perf_counter()
    n_crops = 0
    for (x0, y0, c) in crops:
        ps = [torch.tensor(a, dtype=torch.float64, requires_grad=True) for a in sc.arrays()]
        img = oracle.render.render(*ps, sc.sh_degree, c, st)
        tgt = torch.tensor(target[:, y0:y0 + size, x0:x0 + size], dtype=torch.float64)
        loss = (img - tgt).abs().mean()
        loss.backward()
        n_crops += 1
        if n_crops >= 2 and time.perf_counter() - t0 >= min_seconds:
            break
    dt = time.perf_counter() - t0
    per_px = dt / (n_crops * size * size)
    frame_ms = per_px * cam.width * cam.height * 1e3
    cpu_model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            cpu_model = next(ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name"))
    except (OSError, StopIteration):
        pass
    return dict(value=frame_ms, unit="ms/frame (extrapolated)", cores=torch.get_num_threads(),
                cpu_model=cpu_model, kind="oracle",
                sample=f"{n_crops} seeded {size}x{size} crops, fwd + autograd bwd, {dt:.1f} s "
                       f"total, extrapolated by pixel count to {cam.width}x{cam.height}")


def settings_desc(st):
    return {"tile": [st.tile_w, st.tile_h], "lds_batch": st.lds_batch or st.tile_w * st.tile_h,
            "cost_order": bool(st.cost_order), "tile_cull": bool(st.tile_cull),
            "persistent": bool(st.persistent)}


def tune(params, sc, cams, st, args):
    from paper_2410_08129_amd import autotune
    if args.tile_cull != "auto":
        st = dataclasses.replace(st, tile_cull=(args.tile_cull == "on"))
    if args.schedule:
        st = autotune.apply(st, autotune.by_name(args.schedule))
        return st, {"mode": "fixed", "best": args.schedule}
    if args.tile:
        st.tile_w = st.tile_h = args.tile
        return st, {"mode": "fixed"}
    st2, rep = autotune.tune(params, sc.sh_degree, cams, st,
                             cull_choices=None if args.tile_cull == "auto" else (st.tile_cull,))
    log(f"bench: autotune -> {settings_desc(st2)}")
    return st2, rep


def run_single(args):
    import numpy as np
    import torch

    from paper_2410_08129_amd import htgs, pmc, scenes

    log(f"bench: workload {args.workload}, generating scene")
    sc, cams, st, desc = workload(args.workload)
    cam = cams[0]
    dev = torch.device("cuda:0")
    params = [torch.tensor(a, device=dev) for a in sc.arrays()]
    st, tune_rep = tune(params, sc, [cam], st, args)
    # the backward writes the gradients (no separate clearing pass)
    st = dataclasses.replace(st, grad_overwrite=True)
    target = torch.tensor(scenes.smooth_target(cam.height, cam.width), device=dev)
    n_inst = htgs.count_instances(params, sc.sh_degree, [cam], st)
    ws = htgs.alloc_workspace(sc.n, [cam], st, n_inst, dev)
    state = torch.empty(htgs.state_bytes([cam], st) // 4, dtype=torch.float32, device=dev)
    img = torch.empty((3, cam.height, cam.width), dtype=torch.float32, device=dev)
    gimg = torch.empty_like(img)
    grads = [torch.zeros_like(p) for p in params]
    inv_n = 1.0 / img.numel()
    log(f"bench: {sc.n} Gaussians, {n_inst} instances, ws {ws.numel() / 2**20:.0f} MiB")

    def step():
        frame = htgs.forward(params, sc.sh_degree, [cam], st, ws=ws, state=state, images=[img])
        if args.forward_only:
            return
        torch.sub(img, target, out=gimg)
        gimg.sign_().mul_(inv_n)
        htgs.backward(params, frame, [gimg], grads=grads)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    flags, _, n_frag = htgs.read_status(ws, fragments=True)
    if flags:
        raise SystemExit(f"status flags {flags} after warm-up")
    log(f"bench: warm-up done, {n_frag} fragments")

    htgs.profile_enable(True)
    htgs.profile_read()
    # an event between steps on the stream the library launches on (the
    # current stream) gives the per-step spread
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    evs[0].record()
    for i in range(args.steps):
        step()
        evs[i + 1].record()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = htgs.profile_read()
    htgs.profile_enable(False)
    ms_step = (t1 - t0) * 1e3 / args.steps
    per_step = np.array([evs[i].elapsed_time(evs[i + 1]) for i in range(args.steps)])
    spread = dict(median=round(float(np.median(per_step)), 4),
                  p10=round(float(np.percentile(per_step, 10)), 4),
                  p90=round(float(np.percentile(per_step, 90)), 4),
                  mean=round(float(per_step.mean()), 4))
    log(f"bench: {args.steps} steps, {ms_step:.3f} ms/step, per-step events {spread}")

    # Algorithmic work of the rasterizer: candidate pairs from the tile lists.
    keys, _, _, _ = htgs.export_bins(params, sc.sh_degree, [cam], st, ws)
    tiles_x = (cam.width + st.tile_w - 1) // st.tile_w
    tiles_y = (cam.height + st.tile_h - 1) // st.tile_h
    pw = np.minimum(st.tile_w, cam.width - np.arange(tiles_x) * st.tile_w)
    ph = np.minimum(st.tile_h, cam.height - np.arange(tiles_y) * st.tile_h)
    tile_px = (ph[:, None] * pw[None, :]).reshape(-1)
    per_tile = np.bincount(keys.astype(np.int64), minlength=tiles_x * tiles_y)
    pairs = int((per_tile * tile_px).sum())

    stages = {k: dict(ms_per_launch=(v[0] / max(v[1], 1)), ms_per_step=v[0] / args.steps)
              for k, v in prof.items() if v[1]}
    work = {"raster_fwd": (FLOPS_PAIR * pairs + FLOPS_FRAG_FWD * n_frag) / 1e12,
            "raster_bwd": (FLOPS_PAIR * pairs + FLOPS_FRAG_BWD * n_frag) / 1e12}
    cands = ("raster_fwd",) if args.forward_only else ("raster_fwd", "raster_bwd")
    dom = max(cands, key=lambda k: stages.get(k, {}).get("ms_per_step", 0.0))
    ach = work[dom] / (stages[dom]["ms_per_launch"] * 1e-3)
    # HBM bytes per launch of that kernel from the stored counter record of
    # this workload, if it was taken on the current kernel sources
    kmax = next(k for k in (1, 2, 4, 8, 16, 32) if k >= max(st.K, 1))
    exact = "true" if st.K == kmax else "false"
    persist = "true" if st.persistent else "false"
    if dom == "raster_bwd":
        key = f"k_raster_bwd<{kmax}, {st.tile_w}, {st.tile_h}, {exact}, {persist}>"
    else:
        bm = 2 if st.lds_batch == 2 * st.tile_w * st.tile_h else 1
        key = f"k_raster_fwd<{kmax}, {st.tile_w}, {st.tile_h}, {bm}, {exact}, {persist}>"
    tr = pmc.traffic_for(os.path.join(ROOT, "profiles", f"hbm_traffic_{args.workload}.json"), key)
    roofline = dict(kernel=dom, bound="alu", achieved=round(ach, 3),
                    peak=round(FP32_PEAK_TFLOPS, 1), unit="TFLOP/s",
                    frac=round(ach / FP32_PEAK_TFLOPS, 4),
                    traffic=(round(tr["total"]) if tr else None))
    if tr:
        roofline["traffic_unit"] = "bytes/launch"
    # HBM-bound front end (algorithmic bytes): per sort pass (its count,
    # scan and scatter launches), keys and values read and written once;
    # binning + sort as a whole, B_bin =
    # 8 N + I [(k+4) emit + k histogram + 2 P (k+4) sort + k ranges] + 8 tiles;
    # preprocess reads the parameters and writes record, rect and offset.
    n_tiles = tiles_x * tiles_y
    key_bits = max(1, (n_tiles - 1).bit_length())
    passes = (key_bits + 7) // 8
    kb = 2 if key_bits <= 16 else 4
    sort_bytes_pass = n_inst * 2 * (kb + 4)
    b_bin = 8 * sc.n + n_inst * ((kb + 4) + kb + 2 * passes * (kb + 4) + kb) + 8 * n_tiles
    b_pre = sc.n * (4 * (11 + 3 * (sc.sh_degree + 1) ** 2) + 4 * 32 + 16 + 4)
    binning = None
    if "sort" in stages:
        ms_pass = stages["sort"]["ms_per_step"] / passes
        gbs = sort_bytes_pass / (ms_pass * 1e-3) / 1e9
        t_front = sum(stages[k]["ms_per_step"] for k in ("preprocess", "sort", "ranges")
                      if k in stages)
        gbs_front = (b_bin + b_pre) / (t_front * 1e-3) / 1e9
        t_sort = sum(stages[k]["ms_per_step"] for k in ("sort", "ranges") if k in stages)
        binning = dict(
            kernel="sort_pass", bound="hbm", achieved=round(gbs, 1), peak=HBM_PEAK_GBS,
            unit="GB/s", frac=round(gbs / HBM_PEAK_GBS, 4), bytes_per_pass=sort_bytes_pass,
            ms_per_pass=round(ms_pass, 4),
            sort_and_ranges=dict(ms=round(t_sort, 4), bytes=n_inst * (2 * passes * (kb + 4) + kb)
                                 + 8 * n_tiles),
            front_end=dict(stages="preprocess+emit+sort+ranges", ms=round(t_front, 4),
                           bytes=b_bin + b_pre, achieved=round(gbs_front, 1),
                           frac=round(gbs_front / HBM_PEAK_GBS, 4)))
    out = {
        "metric": "fwd+bwd ms/frame at 1080p & 1M Gaussians",
        "value": round(ms_step, 4),
        "unit": "ms/frame",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": desc, "gaussians": sc.n, "width": cam.width,
                   "height": cam.height, "K": st.K, **settings_desc(st)},
        "roofline": roofline,
        "binning_roofline": binning,
        "ms_per_step_events": spread,
        "stages_ms_per_step": {k: round(v["ms_per_step"], 4) for k, v in stages.items()},
        "instances": n_inst,
        "fragments": n_frag,
        "candidate_pairs": pairs,
        "gaussian_pixels_per_s": sc.n * cam.width * cam.height / (ms_step * 1e-3),
        "candidate_pairs_per_s": pairs / (ms_step * 1e-3),
        "passes": pass_split(stages, sc.n * cam.width * cam.height, pairs),
        "autotune": tune_rep,
    }
    if args.workload != "1080p" or args.forward_only:
        out["metric"] = f"{'fwd' if args.forward_only else 'fwd+bwd'} ms/frame ({args.workload})"
    if args.calibrate_copy:
        # an elementwise kernel (not a DMA copy) so the HBM counters see it
        src = torch.ones(64 << 20, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
        out["copy_calibration_bytes"] = {"read": src.numel() * 4, "write": dst.numel() * 4}
        del src, dst
    del ws, state, grads
    if not args.no_variants and not args.forward_only:
        out["variants"] = run_variants(args, params, sc, cam, st, target)
    del params
    torch.cuda.empty_cache()
    return out, (sc, cam, st)


def pass_split(stages, gauss_px, pairs):
    """Forward and backward apart: the summed HIP-event times of their
    stages per step (no loss kernels, no gaps between launches) and the
    Gaussian x pixel and candidate-pair rates over them."""
    split = {}
    for name, ks in (("fwd", ("fill", "preprocess", "sort", "ranges", "raster_fwd")),
                     ("bwd", ("raster_bwd", "preprocess_bwd"))):
        t = sum(stages[k]["ms_per_step"] for k in ks if k in stages)
        if t > 0:
            split[name] = dict(ms=round(t, 4), stages=list(ks),
                               gaussian_pixels_per_s=gauss_px / (t * 1e-3),
                               candidate_pairs_per_s=pairs / (t * 1e-3))
    return split


def run_variants(args, params, sc, cam, st0, target, steps=10, warmup=3):
    """Other blending modes on the same frame and schedule: hybrid
    transparency with K = 8, 16, 32 (fwd+bwd and forward only), inference
    without the tail (forward), and sorted alpha blending with the early
    stop (forward, and fwd+bwd); each with its own workspace, timed over
    `steps`."""
    import torch

    from paper_2410_08129_amd import htgs

    dev = params[0].device
    out = {}

    def one(name, st, backward):
        n_inst = htgs.count_instances(params, sc.sh_degree, [cam], st)
        ws = htgs.alloc_workspace(sc.n, [cam], st, n_inst, dev)
        state = torch.empty(htgs.state_bytes([cam], st) // 4, dtype=torch.float32, device=dev)
        img = torch.empty((3, cam.height, cam.width), dtype=torch.float32, device=dev)
        gimg = torch.empty_like(img)
        grads = [torch.zeros_like(p) for p in params]

        def step():
            fr = htgs.forward(params, sc.sh_degree, [cam], st, ws=ws, state=state, images=[img])
            if backward:
                torch.sub(img, target, out=gimg)
                gimg.sign_().mul_(1.0 / img.numel())
                htgs.backward(params, fr, [gimg], grads=grads)

        for _ in range(warmup):
            step()
        torch.cuda.synchronize()
        flags, _, n_frag = htgs.read_status(ws, fragments=True)
        htgs.profile_enable(True)
        htgs.profile_read()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            step()
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
        prof = htgs.profile_read()
        htgs.profile_enable(False)
        out[name] = dict(ms_per_step=round(ms, 4), pass_="fwd+bwd" if backward else "fwd",
                         K=st.K, instances=n_inst, fragments=n_frag, status_flags=flags,
                         stages_ms={k: round(v[0] / steps, 4) for k, v in prof.items() if v[1]})
        log(f"bench: variant {name}: {ms:.3f} ms")
        del ws, state, grads

    for K in (8, 16, 32):
        st = dataclasses.replace(st0, K=K)
        if K > 16 and st.tile_w * st.tile_h > 128:
            st = dataclasses.replace(st, tile_w=8, tile_h=8, lds_batch=0)
        one(f"ht_K{K}_fwd_bwd", st, True)
        one(f"ht_K{K}_fwd", st, False)
    one("no_tail_K8_fwd", dataclasses.replace(st0, K=8, no_tail=True, grad_overwrite=False), False)
    one("sorted_fwd", dataclasses.replace(st0, sorted_blend=True, grad_overwrite=False), False)
    one("sorted_fwd_bwd", dataclasses.replace(st0, sorted_blend=True), True)
    for v in out.values():
        v["pass"] = v.pop("pass_")
    return out


def run_multiview(args, steps=3, warmup=1):
    """Plain (16 sequential single-view fwd+bwd calls, no graph) vs batched
    (one hipGraph replay of the batched fwd+bwd); same kernels, same
    accuracy (batched gradient = sum of per-view gradients)."""
    import torch

    from paper_2410_08129_amd import htgs, scenes

    log("bench: multiview, generating 3M-Gaussian scene")
    sc, cams, st, desc = workload("multiview")
    dev = torch.device("cuda:0")
    params = [torch.tensor(a, device=dev) for a in sc.arrays()]
    st, tune_rep = tune(params, sc, cams, st, args)
    targets = [torch.tensor(scenes.smooth_target(c.height, c.width, seed=1 + v), device=dev)
               for v, c in enumerate(cams)]
    imgs = [torch.empty((3, c.height, c.width), dtype=torch.float32, device=dev) for c in cams]
    gimgs = [torch.empty_like(im) for im in imgs]

    # plain: one workspace and state sized for the largest view, reused
    counts = [htgs.count_instances(params, sc.sh_degree, [c], st) for c in cams]
    big = max(range(len(cams)), key=lambda v: cams[v].width * cams[v].height)
    ws1 = htgs.alloc_workspace(sc.n, [cams[big]], st, max(counts), dev)
    st1 = torch.empty(htgs.state_bytes([cams[big]], st) // 4, dtype=torch.float32, device=dev)
    grads_p = [torch.zeros_like(p) for p in params]

    st_over = dataclasses.replace(st, grad_overwrite=True)

    def plain_step():
        # the first view writes the gradients, the others add to them
        for v, c in enumerate(cams):
            fr = htgs.forward(params, sc.sh_degree, [c], st_over if v == 0 else st, ws=ws1,
                              state=st1, images=[imgs[v]])
            torch.sub(imgs[v], targets[v], out=gimgs[v])
            gimgs[v].sign_().mul_(1.0 / imgs[v].numel())
            htgs.backward(params, fr, [gimgs[v]], grads=grads_p)

    n_b = htgs.count_instances(params, sc.sh_degree, cams, st)
    wsb = htgs.alloc_workspace(sc.n, cams, st, n_b, dev)
    stb = torch.empty(htgs.state_bytes(cams, st) // 4, dtype=torch.float32, device=dev)
    grads_b = [torch.zeros_like(p) for p in params]
    imgs_b = [torch.empty_like(im) for im in imgs]
    gimgs_b = [torch.empty_like(im) for im in imgs]
    log(f"bench: multiview {len(cams)} views, {sum(counts)} instances (per view), "
        f"{n_b} (batched), batched ws {wsb.numel() / 2**30:.1f} GiB")

    def batched_step():
        fr = htgs.forward(params, sc.sh_degree, cams, st_over, ws=wsb, state=stb, images=imgs_b)
        for v in range(len(cams)):
            torch.sub(imgs_b[v], targets[v], out=gimgs_b[v])
            gimgs_b[v].sign_().mul_(1.0 / imgs_b[v].numel())
        htgs.backward(params, fr, gimgs_b, grads=grads_b)

    for _ in range(warmup):
        plain_step()
        batched_step()
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        batched_step()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        batched_step()
    torch.cuda.synchronize()

    def timed(fn):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / steps

    ms_plain = timed(plain_step)
    ms_batched = timed(graph.replay)
    # stage split of one eager batched step
    htgs.profile_enable(True)
    htgs.profile_read()
    batched_step()
    torch.cuda.synchronize()
    stages = {k: round(v[0], 3) for k, v in htgs.profile_read().items() if v[1]}
    htgs.profile_enable(False)
    flags, _ = htgs.read_status(wsb)
    rel = {}
    for name, a, b in zip(("means", "log_scales", "quats", "opacity_logits", "sh"),
                          grads_b, grads_p):
        rel[name] = float((a - b).norm() / b.norm().clamp_min(1e-30))
    img_err = max(float((a - b).abs().max()) for a, b in zip(imgs_b, imgs))
    log(f"bench: multiview plain {ms_plain:.2f} ms, batched {ms_batched:.2f} ms")
    out = dict(workload=desc, views=[[c.width, c.height] for c in cams], steps=steps,
               plain_ms_per_step=round(ms_plain, 3), batched_ms_per_step=round(ms_batched, 3),
               speedup=round(ms_plain / ms_batched, 3), batched_stages_ms=stages,
               status_flags=flags,
               batched_vs_plain_image_max_abs=img_err, batched_vs_plain_grad_rel=rel,
               instances=n_b, settings=settings_desc(st), autotune=tune_rep)
    del wsb, ws1, stb, st1, params, grads_p, grads_b
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="1080p")
    ap.add_argument("--tile", type=int, default=0, help="fixed tile size (8 or 16), no autotune")
    ap.add_argument("--tile-cull", choices=("auto", "on", "off"), default="auto",
                    help="exact tile culling of small screen boxes (auto: the autotuner decides)")
    ap.add_argument("--schedule", default="",
                    help="fixed schedule by autotune name (e.g. tile8x8_batch1x_xcd_cull_queue)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-multiview", action="store_true")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the other blending modes (K sweep, no tail, sorted)")
    ap.add_argument("--forward-only", action="store_true")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a plain 256 MiB elementwise copy (reference for HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the renderer runs on a single MI355X).", file=sys.stderr)
        sys.exit(2)

    if args.workload == "multiview":
        mv = run_multiview(args, steps=max(1, args.steps // 5), warmup=1)
        out = {"metric": "batched vs plain speedup (16 views, 3M Gaussians)",
               "value": mv["speedup"], "unit": "x", "n_gpus": 1, "steps": mv["steps"],
               "warmup": 1, "ms_per_step": mv["batched_ms_per_step"], "higher_is_better": True,
               "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
               "config": {"workload": mv["workload"]}, "multiview": mv}
        print(json.dumps(out), flush=True)
        return

    out, (sc, cam, st) = run_single(args)
    if not args.no_multiview and args.workload == "1080p" and not args.forward_only:
        out["multiview"] = run_multiview(args)
    if not args.no_cpu_baseline:
        log("bench: timing the CPU oracle on a bounded sample")
        out["cpu_baseline"] = cpu_baseline(sc, cam, st)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
