"""ctypes binding of ``libhtgs.so`` (C ABI in ``include/htgs.h``) and the
``torch.autograd.Function`` wrapper.

Argument marshalling only: PyTorch provides device memory and the stream;
every step of the renderer runs in the library's HIP kernels. If the library
is not built, every entry point raises; there is no other implementation.
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhtgs.so")

HTGS_OK = 0
HTGS_STATUS_OVERFLOW = 1
HTGS_FLAG_COST_ORDER = 1
HTGS_FLAG_GRAD_OVERWRITE = 2
HTGS_FLAG_TILE_CULL = 4
HTGS_FLAG_PERSISTENT = 8
HTGS_FLAG_NO_TAIL = 16
HTGS_FLAG_BAKED = 32
HTGS_FLAG_SORTED = 64
MAX_VIEWS = 16

EXPORTED = (
    "htgs_workspace_bytes", "htgs_state_bytes", "htgs_count_instances",
    "htgs_render_forward", "htgs_render_backward", "htgs_render_forward_batched",
    "htgs_render_backward_batched", "htgs_read_status", "htgs_debug_export_bins",
    "htgs_strerror", "htgs_version", "htgs_profile_enable", "htgs_profile_read",
    "htgs_debug_fragment_counts", "htgs_opacity_decay",
    "htgs_render_forward_noalloc",
)
STAGES = ("fill", "preprocess", "sort", "ranges", "raster_fwd", "raster_bwd", "reduce",
          "preprocess_bwd", "depth_sort")


class HTGSError(RuntimeError):
    pass


class Gaussians(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("sh_degree", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("means", ctypes.c_void_p), ("log_scales", ctypes.c_void_p),
                ("quats", ctypes.c_void_p), ("opacity_logits", ctypes.c_void_p),
                ("sh", ctypes.c_void_p), ("filter_var", ctypes.c_void_p)]


class Camera(ctypes.Structure):
    _fields_ = [("world_to_cam", ctypes.c_float * 12), ("fx", ctypes.c_float),
                ("fy", ctypes.c_float), ("cx", ctypes.c_float), ("cy", ctypes.c_float),
                ("width", ctypes.c_int32), ("height", ctypes.c_int32),
                ("z_near", ctypes.c_float), ("reserved", ctypes.c_int32)]


class Config(ctypes.Structure):
    _fields_ = [("K", ctypes.c_int32), ("tau_alpha", ctypes.c_float),
                ("tau_core", ctypes.c_float), ("alpha_max", ctypes.c_float),
                ("bg", ctypes.c_float * 3), ("tile_w", ctypes.c_int32),
                ("tile_h", ctypes.c_int32), ("lds_batch", ctypes.c_int32),
                ("flags", ctypes.c_uint32), ("tau_T", ctypes.c_float)]


class Grads(ctypes.Structure):
    _fields_ = [("means", ctypes.c_void_p), ("log_scales", ctypes.c_void_p),
                ("quats", ctypes.c_void_p), ("opacity_logits", ctypes.c_void_p),
                ("sh", ctypes.c_void_p), ("mean_grad_stat", ctypes.c_void_p),
                ("visible_count", ctypes.c_void_p)]


_lib = None


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise HTGSError(f"{LIB_PATH} is missing: build it with "
                        "`python -m paper_2410_08129_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER
    i32, i64, vp = ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p
    L.htgs_workspace_bytes.argtypes = [i64, P(Camera), i32, P(Config), i64, P(i64)]
    L.htgs_state_bytes.argtypes = [P(Camera), i32, P(Config), P(i64)]
    L.htgs_count_instances.argtypes = [P(Gaussians), P(Camera), i32, P(Config), vp, i64, P(i64), vp]
    L.htgs_render_forward.argtypes = [P(Gaussians), P(Camera), P(Config), vp, i64, vp, vp, vp]
    L.htgs_render_forward_noalloc.argtypes = [P(Gaussians), P(Camera), P(Config), vp, vp, vp]
    L.htgs_render_backward.argtypes = [P(Gaussians), P(Camera), P(Config), vp, i64, vp, vp,
                                       P(Grads), vp]
    L.htgs_render_forward_batched.argtypes = [P(Gaussians), P(Camera), i32, P(Config), vp, i64,
                                              vp, P(vp), vp]
    L.htgs_render_backward_batched.argtypes = [P(Gaussians), P(Camera), i32, P(Config), vp, i64,
                                               vp, P(vp), P(Grads), vp]
    L.htgs_read_status.argtypes = [vp, i64, P(ctypes.c_uint32), P(i64), P(i64), vp]
    L.htgs_profile_enable.argtypes = [ctypes.c_int]
    L.htgs_profile_read.argtypes = [P(ctypes.c_double), P(i64), i32]
    L.htgs_debug_export_bins.argtypes = [P(Gaussians), P(Camera), i32, P(Config), vp, i64, vp, vp,
                                         i64, vp, P(i64), vp]
    L.htgs_opacity_decay.argtypes = [vp, i64, ctypes.c_double, vp]
    L.htgs_debug_fragment_counts.argtypes = [vp, i64, P(i64), P(i64), vp]
    L.htgs_strerror.argtypes = [ctypes.c_int]
    L.htgs_strerror.restype = ctypes.c_char_p
    L.htgs_version.argtypes = []
    for name in EXPORTED:
        if name not in ("htgs_strerror",):
            getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def check(code: int, what: str = ""):
    if code != HTGS_OK:
        msg = lib().htgs_strerror(code).decode()
        raise HTGSError(f"{what}: {msg} ({code})")


# ---------------------------------------------------------------------------
# Struct builders
# ---------------------------------------------------------------------------

def camera_struct(cam) -> Camera:
    c = Camera()
    w2c = [float(x) for x in list(cam.world_to_cam.reshape(-1))]
    c.world_to_cam = (ctypes.c_float * 12)(*w2c)
    c.fx, c.fy, c.cx, c.cy = float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy)
    c.width, c.height = int(cam.width), int(cam.height)
    c.z_near = float(cam.z_near)
    return c


def cameras_array(cams):
    arr = (Camera * len(cams))()
    for i, cam in enumerate(cams):
        arr[i] = camera_struct(cam)
    return arr


def config_struct(st) -> Config:
    c = Config()
    c.K = int(st.K)
    c.tau_alpha, c.tau_core, c.alpha_max = float(st.tau_alpha), float(st.tau_core), float(st.alpha_max)
    c.bg = (ctypes.c_float * 3)(*[float(b) for b in st.bg])
    c.tile_w, c.tile_h = int(st.tile_w), int(st.tile_h)
    c.lds_batch = int(getattr(st, "lds_batch", 0))
    c.flags = ((HTGS_FLAG_COST_ORDER if getattr(st, "cost_order", False) else 0)
               | (HTGS_FLAG_GRAD_OVERWRITE if getattr(st, "grad_overwrite", False) else 0)
               | (HTGS_FLAG_TILE_CULL if getattr(st, "tile_cull", False) else 0)
               | (HTGS_FLAG_PERSISTENT if getattr(st, "persistent", False) else 0)
               | (HTGS_FLAG_NO_TAIL if getattr(st, "no_tail", False) else 0)
               | (HTGS_FLAG_BAKED if getattr(st, "baked", False) else 0)
               | (HTGS_FLAG_SORTED if getattr(st, "sorted_blend", False) else 0))
    c.tau_T = float(getattr(st, "tau_T", 0.0))
    return c


def _dev_f32(t: torch.Tensor, name: str) -> torch.Tensor:
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float32):
        raise HTGSError(f"{name} must be a float32 tensor on a HIP device")
    return t.contiguous()


def gaussians_struct(means, log_scales, quats, opacity_logits, sh, sh_degree, filter_var=None):
    """The htgs_gaussians struct and the (contiguous) tensors it points to;
    ``filter_var`` is the optional [n] variance of the 3D filter."""
    ts = [_dev_f32(means, "means"), _dev_f32(log_scales, "log_scales"), _dev_f32(quats, "quats"),
          _dev_f32(opacity_logits, "opacity_logits"), _dev_f32(sh, "sh")]
    n = ts[0].shape[0]
    nb = (int(sh_degree) + 1) ** 2
    shapes = [(n, 3), (n, 3), (n, 4), (n,), (n, nb, 3)]
    for t, s, nm in zip(ts, shapes, ("means", "log_scales", "quats", "opacity_logits", "sh")):
        if tuple(t.shape) != s:
            raise HTGSError(f"{nm} has shape {tuple(t.shape)}, expected {s}")
    g = Gaussians()
    g.n = n
    g.sh_degree = int(sh_degree)
    g.means, g.log_scales, g.quats, g.opacity_logits, g.sh = (t.data_ptr() for t in ts)
    if filter_var is not None:
        fv = _dev_f32(filter_var, "filter_var")
        if tuple(fv.shape) != (n,):
            raise HTGSError(f"filter_var has shape {tuple(fv.shape)}, expected {(n,)}")
        g.filter_var = fv.data_ptr()
        ts.append(fv)
    return g, ts


def _gstruct(params, sh_degree):
    """gaussians_struct of (means, log-scales, quats, logits, sh[, filter_var])."""
    return gaussians_struct(*params[:5], sh_degree,
                            filter_var=params[5] if len(params) > 5 else None)


def stream_handle(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


# ---------------------------------------------------------------------------
# Thin wrappers of the entry points
# ---------------------------------------------------------------------------

def workspace_bytes(n, cams, st, max_instances) -> int:
    out = ctypes.c_int64()
    arr = cameras_array(cams)
    check(lib().htgs_workspace_bytes(int(n), arr, len(cams), ctypes.byref(config_struct(st)),
                                     int(max_instances), ctypes.byref(out)), "workspace_bytes")
    return out.value


def state_bytes(cams, st) -> int:
    out = ctypes.c_int64()
    arr = cameras_array(cams)
    check(lib().htgs_state_bytes(arr, len(cams), ctypes.byref(config_struct(st)),
                                 ctypes.byref(out)), "state_bytes")
    return out.value


def count_instances(params, sh_degree, cams, st, stream=None) -> int:
    g, keep = _gstruct(params, sh_degree)
    arr = cameras_array(cams)
    ws_b = workspace_bytes(g.n, cams, st, 0)
    ws = torch.empty(ws_b, dtype=torch.uint8, device=keep[0].device)
    out = ctypes.c_int64()
    check(lib().htgs_count_instances(ctypes.byref(g), arr, len(cams), ctypes.byref(config_struct(st)),
                                     ctypes.c_void_p(ws.data_ptr()), ws_b, ctypes.byref(out),
                                     stream_handle(stream)), "count_instances")
    return out.value


def read_status(ws: torch.Tensor, stream=None, fragments=False):
    flags = ctypes.c_uint32()
    n = ctypes.c_int64()
    nf = ctypes.c_int64()
    check(lib().htgs_read_status(ctypes.c_void_p(ws.data_ptr()), ws.numel(), ctypes.byref(flags),
                                 ctypes.byref(n), ctypes.byref(nf), stream_handle(stream)),
          "read_status")
    if fragments:
        return flags.value, n.value, nf.value
    return flags.value, n.value


def opacity_decay(opacity_logits: torch.Tensor, lam: float = 0.9995, stream=None):
    """In place: logits <- logit(lam * sigmoid(logits)) (Sec. 4.2)."""
    t = _dev_f32(opacity_logits, "opacity_logits")
    if t.data_ptr() != opacity_logits.data_ptr():
        raise HTGSError("opacity_logits must be contiguous")
    check(lib().htgs_opacity_decay(ctypes.c_void_p(t.data_ptr()), t.numel(), float(lam),
                                   stream_handle(stream)), "opacity_decay")
    return opacity_logits


def fragment_counts(ws: torch.Tensor, stream=None):
    """(forward, backward) fragment counts of the last forward on ``ws`` and
    the backwards since."""
    f, b = ctypes.c_int64(), ctypes.c_int64()
    check(lib().htgs_debug_fragment_counts(ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                                           ctypes.byref(f), ctypes.byref(b),
                                           stream_handle(stream)), "fragment_counts")
    return f.value, b.value


def profile_enable(on: bool):
    check(lib().htgs_profile_enable(1 if on else 0), "profile_enable")


def profile_read():
    """{stage: (milliseconds, launches)} since the last read."""
    ms = (ctypes.c_double * len(STAGES))()
    n = (ctypes.c_int64 * len(STAGES))()
    check(lib().htgs_profile_read(ms, n, len(STAGES)), "profile_read")
    return {s: (ms[i], n[i]) for i, s in enumerate(STAGES)}


class Frame:
    """Device buffers of one forward (kept for the matching backward)."""

    def __init__(self, ws, state, images, cams, st, sh_degree):
        self.ws, self.state, self.images = ws, state, images
        self.cams, self.st, self.sh_degree = cams, st, sh_degree


def alloc_workspace(n, cams, st, instances, device, headroom=1.0):
    cap = int(instances * headroom) + 16
    return torch.empty(workspace_bytes(n, cams, st, cap), dtype=torch.uint8, device=device)


def forward(params, sh_degree, cams, st, ws=None, state=None, images=None, stream=None,
            with_state=True):
    """Renders ``cams`` (a list of 1..16 cameras) into float32 [3,H,W] images.
    Sizes the workspace by counting instances first when ``ws`` is None."""
    g, keep = _gstruct(params, sh_degree)
    dev = keep[0].device
    if ws is None:
        ws = alloc_workspace(g.n, cams, st, count_instances(params, sh_degree, cams, st, stream), dev)
    if with_state and state is None:
        state = torch.empty(state_bytes(cams, st) // 4, dtype=torch.float32, device=dev)
    if images is None:
        images = [torch.empty((3, c.height, c.width), dtype=torch.float32, device=dev) for c in cams]
    arr = cameras_array(cams)
    cfg = config_struct(st)
    sp = ctypes.c_void_p(state.data_ptr()) if with_state else ctypes.c_void_p(0)
    if len(cams) == 1:
        code = lib().htgs_render_forward(ctypes.byref(g), arr, ctypes.byref(cfg),
                                         ctypes.c_void_p(ws.data_ptr()), ws.numel(), sp,
                                         ctypes.c_void_p(images[0].data_ptr()), stream_handle(stream))
    else:
        outs = (ctypes.c_void_p * len(cams))(*[im.data_ptr() for im in images])
        code = lib().htgs_render_forward_batched(ctypes.byref(g), arr, len(cams), ctypes.byref(cfg),
                                                 ctypes.c_void_p(ws.data_ptr()), ws.numel(), sp,
                                                 outs, stream_handle(stream))
    check(code, "render_forward")
    return Frame(ws, state, images, cams, st, sh_degree)


def forward_noalloc(params, sh_degree, cam, st, out, status=None, stream=None):
    """Allocation-free inference render of one camera into ``out`` ([3,H,W]
    float32, caller-allocated) with the library's own workspace; ``status``:
    an optional int32 device tensor of one element that receives the status
    flags."""
    g, keep = _gstruct(params, sh_degree)
    out = _dev_f32(out, "out")
    if tuple(out.shape) != (3, cam.height, cam.width):
        raise HTGSError(f"out has shape {tuple(out.shape)}, expected {(3, cam.height, cam.width)}")
    sp = 0
    if status is not None:
        if not (status.is_cuda and status.dtype == torch.int32 and status.numel() >= 1):
            raise HTGSError("status must be an int32 device tensor")
        sp = status.data_ptr()
    arr = cameras_array([cam])
    check(lib().htgs_render_forward_noalloc(ctypes.byref(g), arr, ctypes.byref(config_struct(st)),
                                            ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(sp),
                                            stream_handle(stream)), "render_forward_noalloc")
    return out


def backward(params, frame: Frame, grad_images, grads=None, stream=None, densify=None):
    """Adds dL/dparams for dL/dimages into ``grads`` (zeros if None);
    ``densify``: optional ([n] mean-gradient statistic, [n] visible count)
    float32 tensors that the densification sums are added to."""
    g, keep = _gstruct(params, frame.sh_degree)
    if grads is None:
        grads = [torch.zeros_like(t) for t in keep[:5]]
    gg = Grads()
    gg.means, gg.log_scales, gg.quats, gg.opacity_logits, gg.sh = (t.data_ptr() for t in grads)
    if densify is not None:
        stat, cnt = (_dev_f32(t, "densify") for t in densify)
        if stat.shape != (g.n,) or cnt.shape != (g.n,):
            raise HTGSError("densify tensors must have shape [n]")
        gg.mean_grad_stat, gg.visible_count = stat.data_ptr(), cnt.data_ptr()
    gis = [_dev_f32(gi, "grad_rgb") for gi in grad_images]
    arr = cameras_array(frame.cams)
    cfg = config_struct(frame.st)
    if len(frame.cams) == 1:
        code = lib().htgs_render_backward(ctypes.byref(g), arr, ctypes.byref(cfg),
                                          ctypes.c_void_p(frame.ws.data_ptr()), frame.ws.numel(),
                                          ctypes.c_void_p(frame.state.data_ptr()),
                                          ctypes.c_void_p(gis[0].data_ptr()), ctypes.byref(gg),
                                          stream_handle(stream))
    else:
        gptr = (ctypes.c_void_p * len(gis))(*[t.data_ptr() for t in gis])
        code = lib().htgs_render_backward_batched(ctypes.byref(g), arr, len(frame.cams),
                                                  ctypes.byref(cfg),
                                                  ctypes.c_void_p(frame.ws.data_ptr()),
                                                  frame.ws.numel(),
                                                  ctypes.c_void_p(frame.state.data_ptr()), gptr,
                                                  ctypes.byref(gg), stream_handle(stream))
    check(code, "render_backward")
    return grads


def export_bins(params, sh_degree, cams, st, ws, stream=None):
    """Sorted tile keys and Gaussian indices of the last forward (host numpy),
    the instance count, and view 0's tile rects."""
    import numpy as np
    g, keep = _gstruct(params, sh_degree)
    flags, n_inst = read_status(ws, stream)
    keys = np.zeros(max(n_inst, 1), np.uint32)
    vals = np.zeros(max(n_inst, 1), np.uint32)
    rects = np.zeros((max(g.n, 1), 4), np.int32)
    out_n = ctypes.c_int64()
    arr = cameras_array(cams)
    check(lib().htgs_debug_export_bins(ctypes.byref(g), arr, len(cams),
                                       ctypes.byref(config_struct(st)),
                                       ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                                       keys.ctypes.data_as(ctypes.c_void_p),
                                       vals.ctypes.data_as(ctypes.c_void_p), keys.size,
                                       rects.ctypes.data_as(ctypes.c_void_p), ctypes.byref(out_n),
                                       stream_handle(stream)), "debug_export_bins")
    n = min(out_n.value, keys.size)
    return keys[:n], vals[:n], rects[:g.n], flags


def state_planes(frame: Frame, view: int = 0):
    """Copies the per-pixel forward state of one view into named planes
    ([values, H, W]); the state itself is tile-major (see htgs.h)."""
    K = int(frame.st.K)
    tw, th = int(frame.st.tile_w), int(frame.st.tile_h)
    sorted_mode = bool(getattr(frame.st, "sorted_blend", False))
    nval = 7 if sorted_mode else 6 * K + 6

    def tiles(c):
        return (c.width + tw - 1) // tw, (c.height + th - 1) // th

    off = 0
    for c in frame.cams[:view]:
        tx, ty = tiles(c)
        off += nval * tx * ty * tw * th
    cam = frame.cams[view]
    tx, ty = tiles(cam)
    bx, by = tw // 8, th // 8
    blk = frame.state[off: off + nval * tx * ty * tw * th]
    # [tile row, tile col, value, block row, block col, row, col]
    blk = blk.view(ty, tx, nval, by, bx, 8, 8).permute(2, 0, 3, 5, 1, 4, 6)
    blk = blk.reshape(nval, ty * th, tx * tw)[:, :cam.height, :cam.width].contiguous()
    if sorted_mode:
        return dict(T=blk[0], S=blk[1:4], end_pos=blk[4].view(torch.int32),
                    n_blended=blk[5].view(torch.int32), stop_id=blk[6].view(torch.int32))
    return dict(core_ids=blk[:K].view(torch.int32), core_alpha=blk[K:2 * K],
                core_pos=blk[2 * K:3 * K].view(torch.int32),
                core_rgb=blk[3 * K:6 * K].reshape(K, 3, cam.height, cam.width),
                T=blk[6 * K], A=blk[6 * K + 1], S=blk[6 * K + 2: 6 * K + 5], P=blk[6 * K + 5])


# ---------------------------------------------------------------------------
# autograd
# ---------------------------------------------------------------------------

class _Render(torch.autograd.Function):
    @staticmethod
    def forward(ctx, st, cams, sh_degree, filter_var, means, log_scales, quats, opacity_logits,
                sh):
        params = (means, log_scales, quats, opacity_logits, sh)
        full = params if filter_var is None else params + (filter_var,)
        frame = forward(full, sh_degree, cams, st)
        flags, _ = read_status(frame.ws)
        if flags:
            raise HTGSError(f"render_forward status flags {flags}")
        ctx.frame = frame
        ctx.filter_var = filter_var
        ctx.save_for_backward(*params)
        return tuple(frame.images)

    @staticmethod
    def backward(ctx, *grad_images):
        params = tuple(ctx.saved_tensors)
        if ctx.filter_var is not None:
            params = params + (ctx.filter_var,)
        gis = [gi.contiguous() if gi is not None else torch.zeros_like(im)
               for gi, im in zip(grad_images, ctx.frame.images)]
        grads = backward(params, ctx.frame, gis)
        ctx.frame = None
        return (None, None, None, None, *grads)


def render(means, log_scales, quats, opacity_logits, sh, sh_degree, cam, settings,
           filter_var=None):
    """Differentiable render of one camera (or a list of up to 16 cameras,
    returning a list of images). ``filter_var``: optional [n] variance of the
    3D filter (an input, not differentiated)."""
    cams = cam if isinstance(cam, (list, tuple)) else [cam]
    outs = _Render.apply(settings, list(cams), int(sh_degree), filter_var, means, log_scales,
                         quats, opacity_logits, sh)
    return list(outs) if isinstance(cam, (list, tuple)) else outs[0]
