"""Python binding of libvr: bricked ray casting + sort-last compositing on MI355X.

Thin ctypes marshalling over the C ABI declared in ``include/vr.h`` (same
function names).  Every step of the rendering path runs in the HIP kernels of
``lib/libvr.so``; there is no CPU fallback: if the library is missing the
import of the binding fails loudly.  PyTorch supplies device memory (tensors)
and streams only.

Method: Hassan, Fluke & Barnes, "Interactive Visualization of the Largest
Radioastronomy Cubes" (arXiv:1008.0135), Sec. 2 (ray casting), Sec. 2.3
(object-space partitioning), Sec. 2.4 (ray-casting process), Sec. 2.5 (image
composition).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "lib", "libvr.so")

VR_OK = 0
VR_EINVAL = -1
VR_ENOMEM = -2
VR_EHIP = -3
VR_ENONFINITE = -4
VR_ESTATE = -5
VR_EUNSUPPORTED = -6
_NAMES = {0: "VR_OK", -1: "VR_EINVAL", -2: "VR_ENOMEM", -3: "VR_EHIP", -4: "VR_ENONFINITE",
          -5: "VR_ESTATE", -6: "VR_EUNSUPPORTED"}

VR_MODE_DVR = 0
VR_MODE_MIP = 1
VR_ERT_LOCAL = 0
VR_ERT_GLOBAL = 1
VR_BRICK_GRID = 0
VR_BRICK_LONGEST_AXIS = 1
VR_STAGE_SETUP, VR_STAGE_MARCH, VR_STAGE_COMPOSITE, VR_STAGE_BACKWARD, VR_STAGE_BATCH = range(5)
VR_NSTAGES = 5


class VRError(RuntimeError):
    def __init__(self, code, func, msg):
        super().__init__(f"{func}: {_NAMES.get(code, code)}: {msg}")
        self.code = code


class vr_view(C.Structure):
    _fields_ = [("R", C.c_double * 9), ("W", C.c_int32), ("H", C.c_int32), ("extent", C.c_double),
                ("eye_dist", C.c_double)]


class vr_params(C.Structure):
    _fields_ = [("step", C.c_double), ("tau", C.c_double), ("ess", C.c_int32), ("ert_scope", C.c_int32),
                ("mode", C.c_int32), ("ckpt_K", C.c_int32), ("tile", C.c_int32), ("reserved", C.c_int32)]


class vr_brick_spec(C.Structure):
    _fields_ = [("mode", C.c_int32), ("nparts", C.c_int32), ("size", C.c_int64 * 3), ("ghost", C.c_int32),
                ("macrocell", C.c_int32), ("materialize", C.c_int32), ("twin", C.c_int32)]


class vr_brick_desc(C.Structure):
    _fields_ = [("lo", C.c_int64 * 3), ("hi", C.c_int64 * 3), ("closed", C.c_int32 * 3), ("reserved", C.c_int32),
                ("slo", C.c_int64 * 3), ("shi", C.c_int64 * 3), ("vmin", C.c_float), ("vmax", C.c_float)]


class vr_brick_image(C.Structure):
    _fields_ = [("brick", C.c_int32), ("x0", C.c_int32), ("y0", C.c_int32), ("w", C.c_int32), ("h", C.c_int32),
                ("reserved", C.c_int32), ("rgba", C.c_void_p)]


class vr_request(C.Structure):
    _fields_ = [("vol", C.c_void_p), ("view", vr_view), ("tf", C.c_void_p), ("m", C.c_int32),
                ("reserved", C.c_int32), ("vmin", C.c_double), ("vmax", C.c_double), ("out", C.c_void_p)]


class vr_tune_result(C.Structure):
    _fields_ = [("tile", C.c_int32), ("waves_per_cu", C.c_int32), ("ms", C.c_double), ("ms_default", C.c_double),
                ("lds_budget", C.c_int32), ("march_mode", C.c_int32)]


class vr_cell_traffic(C.Structure):
    _fields_ = [("own_bytes", C.c_double), ("union_bytes", C.c_double), ("window_bytes", C.c_double),
                ("line_bytes", C.c_double), ("segment_bytes", C.c_double), ("cells", C.c_double), ("cell_layers", C.c_double),
                ("rays_per_cell", C.c_double), ("Tf", C.c_double), ("Tg", C.c_double), ("axis", C.c_int32),
                ("row_floats", C.c_int32), ("rows", C.c_int32), ("twin", C.c_int32)]


_P = C.c_void_p
_I = C.c_int
_I32 = C.c_int32
_I64 = C.c_int64
_D = C.c_double
_U = C.c_uint64  # uintptr_t stream

_SIGS = {
    "vr_last_error": (C.c_char_p, []),
    "vr_version": (_I, []),
    "vr_params_default": (None, [_P]),
    "vr_create": (_I, [_I, _P]),
    "vr_destroy": (_I, [_P]),
    "vr_set_profiling": (_I, [_P, _I]),
    "vr_stage_times": (_I, [_P, _P, _P]),
    "vr_volume_create": (_I, [_P, _P, _I, _I64, _I64, _I64, _P, _P, _U, _P]),
    "vr_volume_wrap": (_I, [_P, _P, _I64, _I64, _I64, _U, _P]),
    "vr_volume_destroy": (_I, [_P]),
    "vr_volume_minmax": (_I, [_P, _P, _P]),
    "vr_volume_dims": (_I, [_P, _P]),
    "vr_volume_brick": (_I, [_P, _P, _U]),
    "vr_volume_brick_info": (_I, [_P, _P, _P]),
    "vr_volume_macrocell_info": (_I, [_P, _P, _P, _P]),
    "vr_tf_set": (_I, [_P, _P, _I32, _D, _D, _I, _U]),
    "vr_mask_set": (_I, [_P, _P, _I32, _I, _U]),
    "vr_render": (_I, [_P, _P, _P, _I32, _P, _P, _U, _P]),
    "vr_render_bricks": (_I, [_P, _P, _P, _P, _P, _P, _P, _U]),
    "vr_composite": (_I, [_P, _P, _I32, _P, _I32, _I32, _P, _U]),
    "vr_render_backward": (_I, [_P, _P, _P, _P, _P, _P, _I, _U]),
    "vr_state_destroy": (_I, [_P]),
    "vr_state_info": (_I, [_P, _I32, _P, _P, _P]),
    "vr_render_batch": (_I, [_P, _P, _I32, _P, _P, _U]),
    "vr_batch_destroy": (_I, [_P]),
    "vr_autotune": (_I, [_P, _P, _P, _P, _P, _U]),
    "vr_autotune_batch": (_I, [_P, _P, _I32, _P, _P, _P, _U]),
    "vr_batch_tiles": (_I, [_P, _P, _I32, _P]),
    "vr_render_batch_noalloc": (_I, [_P, _P, _I32, _P, _U]),
    "vr_plan_view": (_I, [_P, _P, _P, _P, _P, _P, _P]),
    "vr_count_samples": (_I, [_P, _P, _D, _P]),
    "vr_partition": (_I, [_P, _P, _P, _P]),
    "vr_plan_cells": (_I, [_P, _P, _P, _D, _I32, _I32, _P]),
}

_lib = None


def lib():
    """Load lib/libvr.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"libvr.so not found at {LIB_PATH}: build it with "
                "`python -c 'import __graft_entry__ as g; g.build()'` (hipcc, gfx950)")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def exported_symbols():
    return sorted(_SIGS)


def _check(rc, func):
    if rc != VR_OK:
        msg = lib().vr_last_error()
        raise VRError(rc, func, msg.decode() if msg else "")


def _stream(stream):
    if stream is None:
        import torch
        return int(torch.cuda.current_stream().cuda_stream)
    if hasattr(stream, "cuda_stream"):
        return int(stream.cuda_stream)
    return int(stream)


def _ptr(t):
    """Device (or host) address of a torch tensor / numpy array / int."""
    if t is None:
        return None
    if isinstance(t, int):
        return t
    if hasattr(t, "data_ptr"):
        return t.data_ptr()
    if hasattr(t, "ctypes"):
        return t.ctypes.data
    raise TypeError(type(t))


def make_view(R, W, H, extent=0.0, eye_dist=0.0) -> vr_view:
    """eye_dist 0: orthographic; > 0: perspective with the eye that far from the box centre."""
    v = vr_view()
    flat = [float(x) for row in R for x in row] if hasattr(R[0], "__len__") else [float(x) for x in R]
    for i in range(9):
        v.R[i] = flat[i]
    v.W, v.H, v.extent, v.eye_dist = int(W), int(H), float(extent), float(eye_dist)
    return v


def make_params(step=0.5, tau=0.99, ess=1, ckpt_K=32, tile=0, mode=0, ert_scope=0) -> vr_params:
    """mode: VR_MODE_DVR (emission-absorption) or VR_MODE_MIP (maximum intensity projection);
    ert_scope: VR_ERT_LOCAL (per brick) or VR_ERT_GLOBAL (over the whole ray)."""
    p = vr_params()
    lib().vr_params_default(C.byref(p))
    p.step, p.tau, p.ess, p.ckpt_K, p.tile = float(step), float(tau), int(ess), int(ckpt_K), int(tile)
    p.mode = int(mode)
    p.ert_scope = int(ert_scope)
    return p


def grid_spec(size, materialize=False, macrocell=0, twin=False) -> vr_brick_spec:
    s = vr_brick_spec()
    s.mode = VR_BRICK_GRID
    for i in range(3):
        s.size[i] = int(size[i])
    s.ghost = 1
    s.macrocell = int(macrocell)
    s.materialize = int(bool(materialize))
    s.twin = int(bool(twin))
    return s


def kd_spec(nparts, materialize=False, macrocell=0, twin=False) -> vr_brick_spec:
    s = vr_brick_spec()
    s.mode = VR_BRICK_LONGEST_AXIS
    s.nparts = int(nparts)
    s.ghost = 1
    s.macrocell = int(macrocell)
    s.materialize = int(bool(materialize))
    s.twin = int(bool(twin))
    return s


# ------------------------------------------------------------------ C-ABI wrappers
def vr_version():
    return lib().vr_version()


def vr_create(device=0):
    h = C.c_void_p()
    _check(lib().vr_create(int(device), C.byref(h)), "vr_create")
    return h.value


def vr_destroy(ctx):
    _check(lib().vr_destroy(ctx), "vr_destroy")


def vr_set_profiling(ctx, on=True):
    _check(lib().vr_set_profiling(ctx, int(bool(on))), "vr_set_profiling")


def vr_stage_times(ctx):
    ms = (C.c_double * VR_NSTAGES)()
    n = (C.c_int32 * VR_NSTAGES)()
    _check(lib().vr_stage_times(ctx, ms, n), "vr_stage_times")
    return list(ms), list(n)


def vr_volume_create(ctx, src, dims, on_device=None, sub_origin=None, sub_extent=None, stream=None):
    """Upload a [n3][n2][n1] float32 tensor/array (dims = (n1, n2, n3))."""
    if on_device is None:
        on_device = bool(getattr(src, "is_cuda", False))
    h = C.c_void_p()
    so = (C.c_int64 * 3)(*sub_origin) if sub_origin is not None else None
    se = (C.c_int64 * 3)(*sub_extent) if sub_extent is not None else None
    n1, n2, n3 = (int(d) for d in dims)
    _check(lib().vr_volume_create(ctx, _ptr(src), int(on_device), n1, n2, n3, so, se, _stream(stream), C.byref(h)),
           "vr_volume_create")
    return h.value


def vr_volume_wrap(ctx, dev_tensor, dims, stream=None):
    h = C.c_void_p()
    n1, n2, n3 = (int(d) for d in dims)
    _check(lib().vr_volume_wrap(ctx, _ptr(dev_tensor), n1, n2, n3, _stream(stream), C.byref(h)), "vr_volume_wrap")
    return h.value


def vr_volume_destroy(vol):
    _check(lib().vr_volume_destroy(vol), "vr_volume_destroy")


def vr_volume_minmax(vol):
    a, b = C.c_float(), C.c_float()
    _check(lib().vr_volume_minmax(vol, C.byref(a), C.byref(b)), "vr_volume_minmax")
    return a.value, b.value


def vr_volume_dims(vol):
    n = (C.c_int64 * 3)()
    _check(lib().vr_volume_dims(vol, n), "vr_volume_dims")
    return tuple(n)


def vr_volume_brick(vol, spec, stream=None):
    _check(lib().vr_volume_brick(vol, C.byref(spec), _stream(stream)), "vr_volume_brick")


def vr_volume_brick_info(vol):
    nb = C.c_int32(0)
    _check(lib().vr_volume_brick_info(vol, C.byref(nb), None), "vr_volume_brick_info")
    arr = (vr_brick_desc * max(1, nb.value))()
    _check(lib().vr_volume_brick_info(vol, C.byref(nb), arr), "vr_volume_brick_info")
    return [arr[i] for i in range(nb.value)]


def vr_volume_macrocell_info(vol):
    """(edge, (c1, c2, c3), minmax [c3][c2][c1][2] float32 numpy array or None when edge is 0)."""
    edge = C.c_int32(0)
    cnt = (C.c_int64 * 3)()
    _check(lib().vr_volume_macrocell_info(vol, C.byref(edge), cnt, None), "vr_volume_macrocell_info")
    if edge.value == 0:
        return 0, (0, 0, 0), None
    c1, c2, c3 = cnt[0], cnt[1], cnt[2]
    mm = np.empty((c3, c2, c1, 2), dtype=np.float32)
    _check(lib().vr_volume_macrocell_info(vol, C.byref(edge), cnt, mm.ctypes.data_as(C.c_void_p)),
           "vr_volume_macrocell_info")
    return edge.value, (c1, c2, c3), mm


def vr_mask_set(ctx, mask, stream=None):
    """Spectral-channel weights along axis 3 (numpy or torch, host or device); None removes the mask."""
    if mask is None:
        _check(lib().vr_mask_set(ctx, None, 0, 0, _stream(stream)), "vr_mask_set")
        return
    if hasattr(mask, "is_cuda") and mask.is_cuda:
        m = mask.contiguous().float()
        _check(lib().vr_mask_set(ctx, _ptr(m), int(m.numel()), 1, _stream(stream)), "vr_mask_set")
        return
    a = np.ascontiguousarray(mask, dtype=np.float32).reshape(-1)
    _check(lib().vr_mask_set(ctx, a.ctypes.data_as(C.c_void_p), int(a.size), 0, _stream(stream)), "vr_mask_set")


def vr_tf_set(ctx, tf, vmin=0.0, vmax=0.0, stream=None):
    """tf: [m][4] float32 (numpy array on the host or a torch tensor on either side)."""
    on_dev = bool(getattr(tf, "is_cuda", False))
    m = int(tf.shape[0])
    _check(lib().vr_tf_set(ctx, _ptr(tf), m, float(vmin), float(vmax), int(on_dev), _stream(stream)), "vr_tf_set")


def vr_render(ctx, vol, views, params, out, stream=None, save=False):
    """views: list of vr_view; out: device tensor [nv][H][W][4] float32.  Returns the state handle if save."""
    arr = (vr_view * len(views))(*views)
    st = C.c_void_p()
    _check(lib().vr_render(ctx, vol, arr, len(views), C.byref(params), _ptr(out), _stream(stream),
                           C.byref(st) if save else None), "vr_render")
    return st.value if save else None


def vr_render_bricks(ctx, vol, view, params, capacity=65536, stream=None):
    """Returns (list of vr_brick_image, front-to-back order list)."""
    imgs = (vr_brick_image * capacity)()
    order = (C.c_int32 * capacity)()
    n = C.c_int32(capacity)
    _check(lib().vr_render_bricks(ctx, vol, C.byref(view), C.byref(params), imgs, C.byref(n), order,
                                  _stream(stream)), "vr_render_bricks")
    return [imgs[i] for i in range(n.value)], [order[i] for i in range(n.value)]


def vr_composite(ctx, imgs, order, W, H, out, stream=None):
    n = len(imgs)
    arr = (vr_brick_image * max(1, n))(*imgs)
    o = (C.c_int32 * max(1, n))(*order) if order is not None else None
    _check(lib().vr_composite(ctx, arr, n, o, int(W), int(H), _ptr(out), _stream(stream)), "vr_composite")


def vr_render_backward(ctx, vol, state, grad_out, grad_tf, grad_vol=None, accumulate=False, stream=None):
    _check(lib().vr_render_backward(ctx, vol, state, _ptr(grad_out), _ptr(grad_tf), _ptr(grad_vol),
                                    int(bool(accumulate)), _stream(stream)), "vr_render_backward")


def vr_state_destroy(state):
    _check(lib().vr_state_destroy(state), "vr_state_destroy")


def vr_state_info(state, view=0):
    """(ring layout?, cell layers per checkpoint group, samples per checkpoint) of one view."""
    ring, layers, samples = C.c_int32(), C.c_int32(), C.c_double()
    _check(lib().vr_state_info(state, int(view), C.byref(ring), C.byref(layers), C.byref(samples)),
           "vr_state_info")
    return bool(ring.value), layers.value, samples.value


def vr_render_batch(ctx, reqs, params, cache=None, stream=None):
    """reqs: list of vr_request.  Returns the (possibly new) cache handle."""
    arr = (vr_request * len(reqs))(*reqs)
    h = C.c_void_p(cache)
    _check(lib().vr_render_batch(ctx, arr, len(reqs), C.byref(params), C.byref(h), _stream(stream)),
           "vr_render_batch")
    return h.value


def vr_batch_destroy(b):
    _check(lib().vr_batch_destroy(b), "vr_batch_destroy")


def vr_autotune(ctx, vol, view, params, stream=None):
    r = vr_tune_result()
    _check(lib().vr_autotune(ctx, vol, C.byref(view), C.byref(params), C.byref(r), _stream(stream)), "vr_autotune")
    return r


def vr_autotune_batch(ctx, reqs, params, cache=None, stream=None):
    """Returns (tune result, cache handle)."""
    arr = (vr_request * len(reqs))(*reqs)
    h = C.c_void_p(cache)
    r = vr_tune_result()
    _check(lib().vr_autotune_batch(ctx, arr, len(reqs), C.byref(params), C.byref(h), C.byref(r), _stream(stream)),
           "vr_autotune_batch")
    return r, h.value


def vr_render_batch_noalloc(ctx, reqs, params, stream=None):
    """Batched render that allocates nothing (library-held device scratch)."""
    arr = (vr_request * len(reqs))(*reqs)
    _check(lib().vr_render_batch_noalloc(ctx, arr, len(reqs), C.byref(params), _stream(stream)),
           "vr_render_batch_noalloc")


def vr_batch_tiles(ctx, reqs):
    """Tile width each request of a batch runs with (tuned per size class, else 8)."""
    arr = (vr_request * len(reqs))(*reqs)
    t = (C.c_int32 * max(1, len(reqs)))()
    _check(lib().vr_batch_tiles(ctx, arr, len(reqs), t), "vr_batch_tiles")
    return [int(x) for x in t[:len(reqs)]]


def make_request(vol, R, W, H, tf, vmin, vmax, out, extent=0.0, eye_dist=0.0):
    q = vr_request()
    q.vol = vol
    q.view = make_view(R, W, H, extent, eye_dist)
    q.tf = _ptr(tf)
    q.m = int(tf.shape[0])
    q.vmin, q.vmax = float(vmin), float(vmax)
    q.out = _ptr(out)
    return q


def vr_plan_view(dims, spec, view, capacity=65536, waves=False):
    """Returns (rects, order), or (rects, order, waves) with waves=True."""
    d = (C.c_int64 * 3)(*[int(x) for x in dims])
    rects = (C.c_int32 * (4 * capacity))()
    order = (C.c_int32 * capacity)()
    wv = (C.c_int32 * capacity)() if waves else None
    nb = C.c_int32(capacity)
    _check(lib().vr_plan_view(d, C.byref(spec), C.byref(view), C.byref(nb), rects, order, wv), "vr_plan_view")
    n = nb.value
    out = [tuple(rects[4 * i:4 * i + 4]) for i in range(n)], [order[i] for i in range(n)]
    return out + ([wv[i] for i in range(n)],) if waves else out


def vr_partition(dims, spec):
    d = (C.c_int64 * 3)(*[int(x) for x in dims])
    nb = C.c_int32(0)
    _check(lib().vr_partition(d, C.byref(spec), C.byref(nb), None), "vr_partition")
    arr = (vr_brick_desc * max(1, nb.value))()
    _check(lib().vr_partition(d, C.byref(spec), C.byref(nb), arr), "vr_partition")
    return [arr[i] for i in range(nb.value)]


def vr_plan_cells(dims, spec, view, rays=0.0, kmax=0, tf_entries=0):
    """Window-traffic model of the footprint-cell march for one parallel view
    (host only); returns a vr_cell_traffic."""
    d = (C.c_int64 * 3)(*[int(x) for x in dims])
    out = vr_cell_traffic()
    _check(lib().vr_plan_cells(d, C.byref(spec), C.byref(view), float(rays), int(kmax), int(tf_entries),
                               C.byref(out)), "vr_plan_cells")
    return out


def vr_count_samples(dims, view, step=0.5):
    d = (C.c_int64 * 3)(*[int(x) for x in dims])
    out = C.c_int64()
    _check(lib().vr_count_samples(d, C.byref(view), float(step), C.byref(out)), "vr_count_samples")
    return out.value
