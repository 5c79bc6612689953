"""Schedule options of the HIP path (needs an MI355X): the tile order, the
forward LDS batch depth and the tile shape change only how work is mapped
onto the GPU, never which fragments a pixel blends or in which order; a
hipGraph holding the batched forward + backward replays to the eager
result; the autotuner returns one of its candidates and caches it."""
import dataclasses
import json

import numpy as np
import pytest
import torch

import oracle
from paper_2410_08129_amd import autotune, htgs, scenes
from tests import parity

pytestmark = pytest.mark.gpu


def log(msg):
    print(msg, flush=True)


def to_dev(sc):
    return [torch.tensor(a, device="cuda") for a in sc.arrays()]


def fwd_bwd(params, sh_degree, cams, st, Gs):
    frame = htgs.forward(params, sh_degree, cams, st)
    grads = htgs.backward(params, frame, Gs)
    torch.cuda.synchronize()
    flags, _ = htgs.read_status(frame.ws)
    assert flags == 0, flags
    planes = [htgs.state_planes(frame, v) for v in range(len(cams))]
    return frame, grads, planes


@pytest.fixture(scope="module")
def crop_1080p():
    sc, cams, st = scenes.workload_1080p()
    cam = cams[0].crop(811, 397, 301, 203)       # ragged in both directions at 8x8 and 16x16
    G = torch.tensor(np.random.default_rng(3).normal(0, 1e-3, (3, cam.height, cam.width)),
                     dtype=torch.float32, device="cuda")
    return sc, cam, st, to_dev(sc), G


@pytest.mark.parametrize("tile,lds_batch,cost_order,cull,persist", [
    (8, 128, False, False, False), (8, 0, True, False, False), (8, 128, True, False, False),
    (16, 0, True, False, False), (8, 0, False, True, False), (16, 0, False, True, False),
    (8, 0, False, False, True), (8, 0, True, False, True), (16, 0, True, False, True),
    ((16, 8), 0, True, False, True),
])
def test_schedule_options_bit_identical(crop_1080p, tile, lds_batch, cost_order, cull, persist):
    sc, cam, st, params, G = crop_1080p
    tw, th = tile if isinstance(tile, tuple) else (tile, tile)
    base = dataclasses.replace(st, tile_w=tw, tile_h=th, lds_batch=0, cost_order=False)
    var = dataclasses.replace(base, lds_batch=lds_batch, cost_order=cost_order, tile_cull=cull,
                              persistent=persist)
    log(f"schedule tile={tile} lds_batch={lds_batch} cost_order={cost_order} cull={cull} "
        f"persistent={persist}")
    f0, g0, p0 = fwd_bwd(params, sc.sh_degree, [cam], base, [G])
    f1, g1, p1 = fwd_bwd(params, sc.sh_degree, [cam], var, [G])
    assert torch.equal(f0.images[0], f1.images[0])
    for k in ("core_ids", "core_alpha", "T", "A", "S", "P"):
        assert torch.equal(p0[0][k], p1[0][k]), k
    for a, b in zip(g0, g1):
        if cull:
            # fewer instances regroup the per-Gaussian sums: equal up to rounding
            assert float((a - b).norm()) <= 1e-5 * max(float(b.norm()), 1e-30)
        else:
            assert torch.equal(a, b)


def test_tile_shape_changes_only_rounding(crop_1080p):
    sc, cam, st, params, G = crop_1080p
    s8 = dataclasses.replace(st, tile_w=8, tile_h=8)
    s16 = dataclasses.replace(st, tile_w=16, tile_h=16)
    f8, g8, p8 = fwd_bwd(params, sc.sh_degree, [cam], s8, [G])
    f16, g16, p16 = fwd_bwd(params, sc.sh_degree, [cam], s16, [G])
    err = float((f8.images[0] - f16.images[0]).abs().max())
    log(f"  8x8 vs 16x16 image max-abs {err:.3g}")
    assert err < 1e-4
    same_core = float((p8[0]['core_ids'] == p16[0]['core_ids']).float().mean())
    assert same_core > 0.999
    for a, b in zip(g8, g16):
        assert float((a - b).norm()) <= 1e-3 * max(float(b.norm()), 1e-30)


def test_graph_replay_matches_eager():
    sc, cams, st = scenes.workload_small()
    views = [cams[0], cams[0].crop(10, 20, 100, 60),
             scenes.look_at((1.5, -1.0, -2.5), (0, 0, 0), (0, -1, 0), 50.0, 90, 70)]
    st = scenes.RenderSettings(K=4, tile_w=8, tile_h=8, cost_order=True, persistent=True)
    params = to_dev(sc)
    n_inst = htgs.count_instances(params, sc.sh_degree, views, st)
    ws = htgs.alloc_workspace(sc.n, views, st, n_inst, torch.device("cuda"))
    state = torch.empty(htgs.state_bytes(views, st) // 4, dtype=torch.float32, device="cuda")
    imgs = [torch.empty((3, v.height, v.width), dtype=torch.float32, device="cuda") for v in views]
    Gs = [torch.tensor(np.random.default_rng(i).normal(0, 1, (3, v.height, v.width)),
                       dtype=torch.float32, device="cuda") for i, v in enumerate(views)]
    grads = [torch.zeros_like(p) for p in params]

    def step():
        for g in grads:
            g.zero_()
        fr = htgs.forward(params, sc.sh_degree, views, st, ws=ws, state=state, images=imgs)
        htgs.backward(params, fr, Gs, grads=grads)

    step()
    torch.cuda.synchronize()
    ref_imgs = [im.clone() for im in imgs]
    ref_grads = [g.clone() for g in grads]
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        step()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        step()
    torch.cuda.synchronize()
    for r in range(4):
        # eager work on the same workspace between replays: the graph must
        # not depend on anything a previous call left behind
        other = htgs.forward(params, sc.sh_degree, [views[(r + 1) % 3]], st, ws=ws)
        torch.cuda.synchronize()
        assert htgs.read_status(other.ws)[0] == 0
        for t in imgs + grads:
            t.fill_(float("nan"))
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        log(f"  replay {r}")
        assert htgs.read_status(ws)[0] == 0
        for a, b in zip(imgs, ref_imgs):
            assert torch.equal(a, b)
        for a, b in zip(grads, ref_grads):
            assert torch.equal(a, b)


def test_autotune_returns_a_candidate_and_caches(tmp_path, monkeypatch):
    sc, cams, st = scenes.workload_small()
    st = scenes.RenderSettings(K=4)
    params = to_dev(sc)
    path = tmp_path / "tune.json"
    monkeypatch.setenv("HTGS_TUNE_CACHE", str(path))
    monkeypatch.setenv("HTGS_TUNE", "search")
    st1, rep = autotune.tune(params, sc.sh_degree, cams, st, steps=2)
    assert rep["mode"] == "search"
    assert tuple(rep["choice"]) in autotune.CANDIDATES
    assert len(rep["ms"]) == len(autotune.CANDIDATES)
    assert all(v > 0 for v in rep["ms"].values())
    cached = json.loads(path.read_text())
    assert len(cached) == 1
    monkeypatch.setenv("HTGS_TUNE", "cache")
    st2, rep2 = autotune.tune(params, sc.sh_degree, cams, st, steps=2)
    assert rep2["mode"] == "cache" and st2 == st1
    # the tuned settings still render to the oracle's image
    frame = htgs.forward(params, sc.sh_degree, cams, st2)
    torch.cuda.synchronize()
    ref, info = oracle.render.render_scene(sc, cams[0], st2, info=True)
    stats = parity.check_image(frame.images[0].cpu().numpy(),
                               htgs.state_planes(frame, 0)['core_ids'].cpu().numpy(),
                               ref.numpy(), info, st2)
    log(f"  tuned {rep['best']}: {stats}")
    assert stats['max_err_clean'] < 1e-4


def test_grad_overwrite_equals_accumulate_from_zero(crop_1080p):
    sc, cam, st, params, G = crop_1080p
    base = dataclasses.replace(st, grad_overwrite=False)
    over = dataclasses.replace(st, grad_overwrite=True)
    frame = htgs.forward(params, sc.sh_degree, [cam], base)
    g_acc = htgs.backward(params, frame, [G])            # into zeros
    g_over = [torch.full_like(p, float("nan")) for p in params]
    frame2 = htgs.forward(params, sc.sh_degree, [cam], over)
    htgs.backward(params, frame2, [G], grads=g_over)
    torch.cuda.synchronize()
    n_zero = int((g_acc[0].abs().sum(1) == 0).sum())
    log(f"  {n_zero} of {sc.n} Gaussians without gradient (written as zeros)")
    assert n_zero > 0
    for a, b in zip(g_acc, g_over):
        assert torch.equal(a, b)


@pytest.mark.parametrize("tile", [8, 16])
def test_tile_cull_drops_only_empty_tiles(tile):
    """With tile culling the lists are a subset of the box lists (same order
    inside each tile), and no dropped (tile, Gaussian) has a float64
    fragment at any pixel centre of its tile."""
    sc, cams, st = scenes.workload_small()
    cam = cams[0]
    st = scenes.RenderSettings(K=4, tile_w=tile, tile_h=tile)
    stc = dataclasses.replace(st, tile_cull=True)
    params = to_dev(sc)
    fp = htgs.forward(params, sc.sh_degree, [cam], st, with_state=False)
    kp, vp, _, _ = htgs.export_bins(params, sc.sh_degree, [cam], st, fp.ws)
    fc = htgs.forward(params, sc.sh_degree, [cam], stc, with_state=False)
    kc, vc, _, _ = htgs.export_bins(params, sc.sh_degree, [cam], stc, fc.ws)
    torch.cuda.synchronize()
    keep = {(int(k), int(v)) for k, v in zip(kc, vc)}
    full = [(int(k), int(v)) for k, v in zip(kp, vp)]
    assert keep <= set(full)
    assert [p for p in full if p in keep] == [(int(k), int(v)) for k, v in zip(kc, vc)]
    dropped = [p for p in full if p not in keep]
    log(f"  tile {tile}: {len(full)} box instances, {len(dropped)} dropped")
    assert len(dropped) > 0
    arrs = [torch.tensor(a) for a in sc.arrays()]
    prep = oracle.render.prepare(*arrs, sc.sh_degree, cam, st, cull=False)
    pos = {int(g): i for i, g in enumerate(prep.idx.numpy())}
    tx_n = (cam.width + tile - 1) // tile
    for key, g in dropped:
        tx, ty = key % tx_n, key // tx_n
        xs, ys = np.meshgrid(np.arange(tx * tile, min(tx * tile + tile, cam.width)),
                             np.arange(ty * tile, min(ty * tile + tile, cam.height)))
        i = pos[g]
        one = oracle.render.Prepared(*(getattr(prep, f.name)[i:i + 1]
                                       for f in dataclasses.fields(prep)))
        frag = oracle.render.evaluate(one, torch.tensor(xs.ravel() + 0.5, dtype=torch.float64),
                                      torch.tensor(ys.ravel() + 0.5, dtype=torch.float64),
                                      st)[2]
        assert not bool(frag.any()), (key, g)
