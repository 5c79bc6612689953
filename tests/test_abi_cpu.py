"""The C-ABI library loads, exports every entry point of include/htgs.h, and
rejects bad arguments on the host before any device work (no GPU needed)."""
import ctypes
import os
import re

import pytest

from paper_2410_08129_amd import htgs, scenes

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "htgs.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(htgs_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_entry_point():
    L = htgs.lib()
    names = _declared()
    assert len(names) >= 11
    for n in names:
        assert hasattr(L, n), n
    assert set(htgs.EXPORTED) == set(names)
    assert L.htgs_version() == 4


def test_strerror_codes():
    L = htgs.lib()
    for code in (0, -1, -2, -3, -4, -5, -6, 7):
        assert isinstance(L.htgs_strerror(code), bytes)
    assert L.htgs_strerror(-2) == b"workspace too small"


def _small():
    sc, cams, st = scenes.workload_small()
    return sc, cams, st


def test_workspace_and_state_sizes():
    sc, cams, st = _small()
    a = htgs.workspace_bytes(sc.n, cams, st, 0)
    b = htgs.workspace_bytes(sc.n, cams, st, 10000)
    c = htgs.workspace_bytes(sc.n, cams, st, 20000)
    assert 0 < a < b < c
    # 16-bit keys: 2 key buffers x 2 B + 2 value buffers x 4 B + 64 B partials
    assert abs((c - b) - 10000 * (4 + 8 + 64)) < 4096
    st8 = scenes.RenderSettings(K=8)
    assert htgs.state_bytes(cams, st8) == (24 * 8 + 24) * 128 * 128
    # the state is tile-major, each tile padded to full size at the image edge
    two = [cams[0], cams[0].crop(0, 0, 50, 30)]
    tw, th = st8.tile_w, st8.tile_h
    padded = ((50 + tw - 1) // tw * tw) * ((30 + th - 1) // th * th)
    assert htgs.state_bytes(two, st8) == (24 * 8 + 24) * (128 * 128 + padded)


@pytest.mark.parametrize("field,value", [
    ("K", 33), ("K", -1), ("tile_w", 12), ("tau_alpha", 0.0), ("alpha_max", 1.0),
    ("flags", 1 << 10), ("lds_batch", 7), ("lds_batch", 512),
])
def test_bad_config_rejected(field, value):
    sc, cams, st = _small()
    cfg = htgs.config_struct(st)
    setattr(cfg, field, value)
    out = ctypes.c_int64()
    arr = htgs.cameras_array(cams)
    assert htgs.lib().htgs_workspace_bytes(sc.n, arr, 1, ctypes.byref(cfg), 0,
                                           ctypes.byref(out)) == -1


def test_large_core_needs_small_tiles():
    sc, cams, st = _small()
    cfg = htgs.config_struct(scenes.RenderSettings(K=20, tile_w=16, tile_h=16))
    out = ctypes.c_int64()
    assert htgs.lib().htgs_workspace_bytes(sc.n, htgs.cameras_array(cams), 1, ctypes.byref(cfg), 0,
                                           ctypes.byref(out)) == -1
    cfg = htgs.config_struct(scenes.RenderSettings(K=20, tile_w=8, tile_h=8))
    assert htgs.lib().htgs_workspace_bytes(sc.n, htgs.cameras_array(cams), 1, ctypes.byref(cfg), 0,
                                           ctypes.byref(out)) == 0
    for (tw, th, k, ok) in [(16, 8, 32, True), (32, 8, 16, True), (32, 8, 17, False),
                            (8, 16, 4, False), (32, 32, 4, False)]:
        cfg = htgs.config_struct(scenes.RenderSettings(K=k, tile_w=tw, tile_h=th))
        code = htgs.lib().htgs_workspace_bytes(sc.n, htgs.cameras_array(cams), 1,
                                               ctypes.byref(cfg), 0, ctypes.byref(out))
        assert code == (0 if ok else -1), (tw, th, k)


def _fake_gaussians(n=10, deg=0):
    g = htgs.Gaussians()
    g.n, g.sh_degree = n, deg
    # never dereferenced: every call below fails its host checks first
    g.means = g.log_scales = g.quats = g.opacity_logits = g.sh = 0x1000
    return g


def test_forward_argument_errors_before_device_work():
    sc, cams, st = _small()
    L = htgs.lib()
    cam = htgs.camera_struct(cams[0])
    cfg = htgs.config_struct(st)
    g = _fake_gaussians()
    fake = ctypes.c_void_p(0x2000)
    # null workspace / output
    assert L.htgs_render_forward(ctypes.byref(g), ctypes.byref(cam), ctypes.byref(cfg), None, 0,
                                 None, fake, None) == -1
    assert L.htgs_render_forward(ctypes.byref(g), ctypes.byref(cam), ctypes.byref(cfg), fake,
                                 1 << 20, None, None, None) == -1
    # workspace too small
    assert L.htgs_render_forward(ctypes.byref(g), ctypes.byref(cam), ctypes.byref(cfg), fake, 64,
                                 None, fake, None) == -2
    # null parameter pointer with n > 0
    g2 = _fake_gaussians()
    g2.quats = None
    assert L.htgs_render_forward(ctypes.byref(g2), ctypes.byref(cam), ctypes.byref(cfg), fake,
                                 1 << 30, None, fake, None) == -1
    # bad SH degree
    g3 = _fake_gaussians(deg=4)
    assert L.htgs_render_forward(ctypes.byref(g3), ctypes.byref(cam), ctypes.byref(cfg), fake,
                                 1 << 30, None, fake, None) == -1
    # bad camera
    bad = htgs.camera_struct(cams[0])
    bad.width = 0
    assert L.htgs_render_forward(ctypes.byref(g), ctypes.byref(bad), ctypes.byref(cfg), fake,
                                 1 << 30, None, fake, None) == -1
    bad = htgs.camera_struct(cams[0])
    bad.fx = float("nan")
    assert L.htgs_render_forward(ctypes.byref(g), ctypes.byref(bad), ctypes.byref(cfg), fake,
                                 1 << 30, None, fake, None) == -1
    # parameter arrays must be 16-byte aligned
    g4 = _fake_gaussians()
    g4.sh = 0x2004
    assert L.htgs_render_forward(ctypes.byref(g4), ctypes.byref(cam), ctypes.byref(cfg), fake,
                                 1 << 30, None, fake, None) == -1


def test_backward_and_batched_argument_errors():
    sc, cams, st = _small()
    L = htgs.lib()
    cfg = htgs.config_struct(st)
    g = _fake_gaussians()
    fake = ctypes.c_void_p(0x2000)
    arr = htgs.cameras_array(cams * 17)
    outs = (ctypes.c_void_p * 17)(*([0x2000] * 17))
    assert L.htgs_render_forward_batched(ctypes.byref(g), arr, 17, ctypes.byref(cfg), fake,
                                         1 << 30, None, outs, None) == -6
    assert L.htgs_render_forward_batched(ctypes.byref(g), arr, 0, ctypes.byref(cfg), fake,
                                         1 << 30, None, outs, None) == -1
    gr = htgs.Grads()
    cam = htgs.camera_struct(cams[0])
    # missing state
    assert L.htgs_render_backward(ctypes.byref(g), ctypes.byref(cam), ctypes.byref(cfg), fake,
                                  1 << 30, None, fake, ctypes.byref(gr), None) == -1
    assert L.htgs_render_backward(ctypes.byref(g), ctypes.byref(cam), ctypes.byref(cfg), fake, 64,
                                  fake, fake, ctypes.byref(gr), None) == -2
    # gradient arrays must be 16-byte aligned
    gr2 = htgs.Grads()
    gr2.means = 0x2008
    assert L.htgs_render_backward(ctypes.byref(g), ctypes.byref(cam), ctypes.byref(cfg), fake,
                                  1 << 30, fake, fake, ctypes.byref(gr2), None) == -1
    # inference without the tail, and baked inputs, have no backward
    for flags in (dict(no_tail=True), dict(baked=True)):
        nt = htgs.config_struct(scenes.RenderSettings(K=4, **flags))
        assert L.htgs_render_backward(ctypes.byref(g), ctypes.byref(cam), ctypes.byref(nt), fake,
                                      1 << 30, fake, fake, ctypes.byref(gr), None) == -1
    # baked inputs already hold any 3D filter
    gf = _fake_gaussians()
    gf.filter_var = 0x3000
    bk = htgs.config_struct(scenes.RenderSettings(K=4, baked=True))
    assert L.htgs_render_forward(ctypes.byref(gf), ctypes.byref(cam), ctypes.byref(bk), fake,
                                 1 << 30, None, fake, None) == -1
    gf.filter_var = 0x3002     # the filter variance array must be 4-byte aligned
    assert L.htgs_render_forward(ctypes.byref(gf), ctypes.byref(cam), ctypes.byref(cfg), fake,
                                 1 << 30, None, fake, None) == -1
    # densification sums must be 4-byte aligned
    gr3 = htgs.Grads()
    gr3.visible_count = 0x2002
    assert L.htgs_render_backward(ctypes.byref(g), ctypes.byref(cam), ctypes.byref(cfg), fake,
                                  1 << 30, fake, fake, ctypes.byref(gr3), None) == -1
    # opacity decay: lambda in (0, 1], no work for n = 0
    assert L.htgs_opacity_decay(fake, 10, ctypes.c_double(1.5), None) == -1
    assert L.htgs_opacity_decay(fake, 10, ctypes.c_double(0.0), None) == -1
    assert L.htgs_opacity_decay(None, 10, ctypes.c_double(0.9), None) == -1
    assert L.htgs_opacity_decay(None, 0, ctypes.c_double(0.9), None) == 0
    assert L.htgs_read_status(None, 0, None, None, None, None) == -1
    assert L.htgs_profile_read(None, None, 0) == -1
    n = ctypes.c_int64()
    assert L.htgs_count_instances(ctypes.byref(g), ctypes.byref(cam), 1, ctypes.byref(cfg), fake,
                                  64, ctypes.byref(n), None) == -2


def test_binding_refuses_cpu_tensors():
    import torch
    sc, cams, st = _small()
    params = [torch.tensor(a) for a in sc.arrays()]
    with pytest.raises(htgs.HTGSError):
        htgs.forward(params, sc.sh_degree, cams, st)


def test_noalloc_forward_argument_errors_before_device_work():
    """The allocation-free forward rejects bad arguments, and scenes whose
    per-splat data alone exceed its fixed workspace, before any device call."""
    sc, cams, st = _small()
    L = htgs.lib()
    cam = htgs.camera_struct(cams[0])
    cfg = htgs.config_struct(st)
    fake = ctypes.c_void_p(0x2000)
    g = _fake_gaussians()
    assert L.htgs_render_forward_noalloc(ctypes.byref(g), ctypes.byref(cam), ctypes.byref(cfg),
                                         None, None, None) == -1
    # misaligned status word
    assert L.htgs_render_forward_noalloc(ctypes.byref(g), ctypes.byref(cam), ctypes.byref(cfg),
                                         fake, ctypes.c_void_p(0x2002), None) == -1
    bad = htgs.camera_struct(cams[0])
    bad.height = -3
    assert L.htgs_render_forward_noalloc(ctypes.byref(g), ctypes.byref(bad), ctypes.byref(cfg),
                                         fake, None, None) == -1
    # 1M Gaussians: ~160 MB of per-splat data, beyond the 64 MiB array
    big = _fake_gaussians(n=1_000_000)
    assert L.htgs_render_forward_noalloc(ctypes.byref(big), ctypes.byref(cam), ctypes.byref(cfg),
                                         fake, None, None) == -7
    assert b"too large" in L.htgs_strerror(-7)
