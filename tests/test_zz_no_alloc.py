"""The allocation-free forward entry point against the regular forward,
through the C ABI (needs an MI355X): two calls in a row on the library's own
workspace, the second with a smaller scene and image, each bit-identical to
htgs_render_forward with a caller workspace."""
import dataclasses

import pytest
import torch

from paper_2410_08129_amd import htgs, scenes

pytestmark = pytest.mark.gpu


def _regular(params, deg, cam, st):
    frame = htgs.forward(params, deg, [cam], st, with_state=False)
    torch.cuda.synchronize()
    flags, n = htgs.read_status(frame.ws)
    assert flags == 0
    return frame.images[0], n


def test_noalloc_forward_matches_regular_forward_twice():
    sc, cams, st = scenes.workload_small()
    st = dataclasses.replace(st, tile_cull=True, cost_order=True)
    params = [torch.tensor(a, device="cuda") for a in sc.arrays()]
    big_cam = cams[0]
    # second call: fewer Gaussians and a smaller, ragged image
    small_params = [p[:1500].contiguous() for p in params]
    small_cam = big_cam.crop(20, 24, 70, 53)
    status = torch.full((1,), -1, dtype=torch.int32, device="cuda")
    for (ps, cam, label) in ((params, big_cam, "4096 Gaussians 128x128"),
                             (small_params, small_cam, "1500 Gaussians 70x53")):
        print(f"noalloc: {label}", flush=True)
        ref, n_inst = _regular(ps, sc.sh_degree, cam, st)
        out = torch.full((3, cam.height, cam.width), float("nan"), device="cuda")
        htgs.forward_noalloc(ps, sc.sh_degree, cam, st, out, status=status)
        torch.cuda.synchronize()
        assert int(status.item()) == 0
        print(f"  instances {n_inst}, max |diff| {float((out - ref).abs().max()):.3g}", flush=True)
        assert torch.equal(out, ref)


def test_noalloc_forward_reports_overflow_and_too_large():
    sc, cams, st = scenes.workload_small()
    # Gaussians whose per-splat data fits but whose instances do not: every
    # copy of the scene covers the frame with 16x16-pixel boxes at 8x8 tiles
    # -> far more instances than the remaining bytes hold
    params = [torch.tensor(a, device="cuda") for a in sc.arrays()]
    reps = 90
    big = [p.repeat((reps,) + (1,) * (p.dim() - 1)).contiguous() for p in params]
    big[1] = (big[1] + 2.5).contiguous()   # larger splats: many tiles each
    st8 = dataclasses.replace(st, tile_w=8, tile_h=8)
    cam = cams[0]
    out = torch.empty((3, cam.height, cam.width), device="cuda")
    status = torch.zeros((1,), dtype=torch.int32, device="cuda")
    htgs.forward_noalloc(big, sc.sh_degree, cam, st8, out, status=status)
    torch.cuda.synchronize()
    assert int(status.item()) & htgs.HTGS_STATUS_OVERFLOW
    huge = [p.repeat((200,) + (1,) * (p.dim() - 1)).contiguous() for p in params]
    with pytest.raises(htgs.HTGSError, match="too large"):
        htgs.forward_noalloc(huge, sc.sh_degree, cam, st8, out, status=status)
