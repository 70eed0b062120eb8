"""FP64 CPU oracle for bricked ray casting + sort-last compositing.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by the smoke check and by the
CPU-baseline leg of the benchmark, never by the product path.  It shares no
code with the HIP implementation; ``vr_oracle.c`` holds the arithmetic (plain
double-precision loops) and this module only marshals numpy arrays into it.

The partition helpers here (regular grid, longest-axis split) are the oracle's
own statement of the object-space partitioning of paper Sec. 2.3.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "vr_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

FLAG_ERT = 1   # early-termination tie: several images are valid (listed in "ties")
FLAG_GEOM = 2  # a sample count or owner decided within rounding of a face

MAXC = 64  # most valid images listed per ray


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=c11",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class View(C.Structure):
    _fields_ = [("R", C.c_double * 9), ("W", C.c_int), ("H", C.c_int), ("extent", C.c_double),
                ("eye_dist", C.c_double)]


class Box(C.Structure):
    _fields_ = [("lo", C.c_double * 3), ("hi", C.c_double * 3), ("closed", C.c_int * 3)]


class Scene(C.Structure):
    _fields_ = [
        ("vol", C.c_void_p), ("n", C.c_int64 * 3), ("tf", C.c_void_p), ("M", C.c_int),
        ("vmin", C.c_double), ("vmax", C.c_double), ("step", C.c_double), ("tau", C.c_double),
        ("nboxes", C.c_int), ("boxes", C.c_void_p), ("grid", C.c_int), ("gb", C.c_int64 * 3),
        ("gnb", C.c_int * 3), ("ert_margin", C.c_double), ("geom_margin", C.c_double),
        ("mode", C.c_int), ("mask", C.c_void_p),
    ]


MODE_DVR = 0
MODE_MIP = 1


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        L = C.CDLL(_LIB)
        _bind(L)
        _lib = L
    return _lib


def _bind(L):
    """Declare the argument types of the oracle library's entry points."""
    P = C.c_void_p
    L.or_render_rays.argtypes = [P, P, C.c_int, P, P, P, C.c_int64, P, P, P, P, C.c_int]
    L.or_render_candidates.argtypes = [P, P, C.c_int, P, P, P, C.c_int64, P, P, P, P, C.c_int, P, P, C.c_int]
    L.or_render_images.argtypes = [P, P, C.c_int, P, P, P, C.c_int]
    L.or_render_grad.argtypes = [P, P, P, P, P, P, C.c_int]
    L.or_minmax.argtypes = [P, C.c_int64, P, P, P, C.c_int]
    L.or_box_minmax.argtypes = [P, P, P, P, P, P]
    L.or_composite.argtypes = [P, C.c_int, C.c_int64, P]
    return L


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


# ---------------------------------------------------------------- partitions
def grid_boxes(dims, bsize):
    """Regular grid of ownership boxes: brick j owns [j b, (j+1) b), the last is closed at n-1.

    ``dims`` = (n1, n2, n3), ``bsize`` = brick size in cells per axis.  Box
    order: axis 1 fastest.  Returns (list of (lo, hi, closed) tuples, counts).
    """
    counts = []
    for n, b in zip(dims, bsize):
        counts.append(max(1, -(-(n - 1) // b)))
    boxes = []
    for k3 in range(counts[2]):
        for k2 in range(counts[1]):
            for k1 in range(counts[0]):
                lo, hi, cl = [], [], []
                for ax, k in enumerate((k1, k2, k3)):
                    n, b, m = dims[ax], bsize[ax], counts[ax]
                    lo.append(k * b)
                    last = k == m - 1
                    hi.append(n - 1 if last else (k + 1) * b)
                    cl.append(1 if last else 0)
                boxes.append((tuple(lo), tuple(hi), tuple(cl)))
    return boxes, tuple(counts)


def kd_boxes(dims, nparts):
    """Longest-axis recursive split (paper Sec. 2.3) into ``nparts`` ownership boxes.

    A box is split across its longest extent (first such axis on ties) into
    floor(p/2) and p - floor(p/2) parts at the integer plane closest to the
    proportional position.  Returned in depth-first (low side first) order.
    """
    out = []

    def rec(lo, hi, cl, p):
        if p == 1:
            out.append((tuple(lo), tuple(hi), tuple(cl)))
            return
        ext = [hi[i] - lo[i] for i in range(3)]
        ax = max(range(3), key=lambda i: (ext[i], -i))
        pl = p // 2
        cut = lo[ax] + int(round(ext[ax] * pl / p))
        cut = min(max(cut, lo[ax] + 1), hi[ax] - 1)
        hl, cll = list(hi), list(cl)
        hl[ax], cll[ax] = cut, 0
        lr = list(lo)
        lr[ax] = cut
        rec(list(lo), hl, cll, pl)
        rec(lr, list(hi), list(cl), p - pl)

    rec([0, 0, 0], [d - 1 for d in dims], [1, 1, 1], nparts)
    return out


# ---------------------------------------------------------------- rendering
def _scene(vol, tf, vmin, vmax, step, tau, bricks, ert_margin, geom_margin, mode=0, mask=None):
    vol = np.ascontiguousarray(vol, dtype=np.float32)
    tf = np.ascontiguousarray(tf, dtype=np.float32).reshape(-1, 4)
    sc = Scene()
    sc.vol = vol.ctypes.data
    sc.n[0], sc.n[1], sc.n[2] = vol.shape[2], vol.shape[1], vol.shape[0]
    sc.tf = tf.ctypes.data
    sc.M = tf.shape[0]
    sc.vmin, sc.vmax, sc.step, sc.tau = float(vmin), float(vmax), float(step), float(tau)
    sc.ert_margin, sc.geom_margin = float(ert_margin), float(geom_margin)
    sc.mode = int(mode)
    keep = [vol, tf]
    if mask is not None:
        mask = np.ascontiguousarray(mask, dtype=np.float32).reshape(-1)
        if mask.shape[0] != vol.shape[0]:
            raise ValueError("mask needs one weight per index along axis 3")
        sc.mask = mask.ctypes.data
        keep.append(mask)
    if bricks is not None:
        dims = (vol.shape[2], vol.shape[1], vol.shape[0])
        if isinstance(bricks, dict) and "grid" in bricks:
            bs = bricks["grid"]
            boxes, counts = grid_boxes(dims, bs)
            sc.grid = 1
            for i in range(3):
                sc.gb[i] = bs[i]
                sc.gnb[i] = counts[i]
        else:
            boxes = bricks["boxes"] if isinstance(bricks, dict) else bricks
        arr = (Box * len(boxes))()
        for j, (lo, hi, cl) in enumerate(boxes):
            for i in range(3):
                arr[j].lo[i], arr[j].hi[i], arr[j].closed[i] = lo[i], hi[i], cl[i]
        sc.nboxes = len(boxes)
        sc.boxes = C.addressof(arr)
        keep.append(arr)
    return sc, keep


def _views(views, W, H, extent, eye_dist=0.0):
    arr = (View * len(views))()
    for j, R in enumerate(views):
        R = np.asarray(R, dtype=np.float64).reshape(9)
        for i in range(9):
            arr[j].R[i] = R[i]
        arr[j].W, arr[j].H, arr[j].extent = int(W), int(H), float(extent)
        arr[j].eye_dist = float(eye_dist)
    return arr


def _ties(sc, vw, nv, rv, ru, rr, nthreads):
    """Every valid image of the given rays (early-termination ties)."""
    n = rv.shape[0]
    cand = np.zeros((n, MAXC, 4), np.float64)
    ncand = np.zeros(n, np.int32)
    if n:
        rc = lib().or_render_candidates(C.byref(sc), vw, nv, _ptr(rv), _ptr(ru), _ptr(rr), n, None, None, None,
                                        None, MAXC, _ptr(cand), _ptr(ncand), int(nthreads))
        if rc != 0:
            raise ValueError("oracle candidates: bad input")
    return cand, ncand


def render(vol, tf, views, W, H, vmin, vmax, step=0.5, tau=0.99, extent=0.0, bricks=None,
           ert_margin=1e-5, geom_margin=1e-9, nthreads=0, mode=MODE_DVR, eye_dist=0.0, mask=None):
    """Render full images.  Returns dict(image [nv][H][W][4] f64, flags [nv][H][W], nsamples, ties).

    ties = dict(index, cand, ncand): for each pixel flagged FLAG_ERT (flat index
    into ``flags``), every valid image (cand[i][:ncand[i]], RGBA) -- one per
    combination of the stopping samples that lie within ``ert_margin`` of tau
    in opacity; ncand = -1 when there are more than MAXC.

    mode=MODE_MIP: maximum intensity projection, (M, M, M, M) per pixel with M the
    largest normalised sample value along the ray (the table is not used).
    eye_dist > 0: perspective camera with the eye at distance eye_dist from the box
    centre (0: orthographic).  mask: optional weight per index along axis 3 (spectral
    channels), multiplying each sample's opacity (MIP: its normalised value)."""
    sc, keep = _scene(vol, tf, vmin, vmax, step, tau, bricks, ert_margin, geom_margin, mode, mask)
    vw = _views(views, W, H, extent, eye_dist)
    nv = len(views)
    img = np.zeros((nv, H, W, 4), np.float64)
    flags = np.zeros((nv, H, W), np.uint8)
    tot = C.c_int64(0)
    rc = lib().or_render_images(C.byref(sc), vw, nv, _ptr(img), _ptr(flags), C.byref(tot), int(nthreads))
    if rc != 0:
        raise ValueError("oracle render: bad input")
    idx = np.flatnonzero((flags & FLAG_ERT) != 0)
    vi, yy, xx = np.unravel_index(idx, flags.shape)
    cand, ncand = _ties(sc, vw, nv, np.ascontiguousarray(vi, np.int32), np.ascontiguousarray(xx, np.int32),
                        np.ascontiguousarray(yy, np.int32), nthreads)
    del keep
    return dict(image=img, flags=flags, nsamples=int(tot.value), ties=dict(index=idx, cand=cand, ncand=ncand))


def render_rays(vol, tf, views, W, H, ray_view, ray_u, ray_v, vmin, vmax, step=0.5, tau=0.99,
                extent=0.0, bricks=None, ert_margin=1e-5, geom_margin=1e-9, nthreads=0, mode=MODE_DVR,
                eye_dist=0.0, mask=None):
    """Render selected rays (view index, pixel u, pixel v).  Returns dict like ``render``
    (``nsamples`` per ray, ``ties.index`` into the ray list) plus ``neval``: samples
    evaluated per ray (each sub-volume's samples up to its own stop)."""
    sc, keep = _scene(vol, tf, vmin, vmax, step, tau, bricks, ert_margin, geom_margin, mode, mask)
    vw = _views(views, W, H, extent, eye_dist)
    rv = np.ascontiguousarray(ray_view, np.int32)
    ru = np.ascontiguousarray(ray_u, np.int32)
    rr = np.ascontiguousarray(ray_v, np.int32)
    n = rv.shape[0]
    img = np.zeros((n, 4), np.float64)
    flags = np.zeros(n, np.uint8)
    ns = np.zeros(n, np.int64)
    ne = np.zeros(n, np.int64)
    rc = lib().or_render_rays(C.byref(sc), vw, len(views), _ptr(rv), _ptr(ru), _ptr(rr), n,
                              _ptr(img), _ptr(flags), _ptr(ns), _ptr(ne), int(nthreads))
    if rc != 0:
        raise ValueError("oracle render_rays: bad input")
    idx = np.flatnonzero((flags & FLAG_ERT) != 0)
    cand, ncand = _ties(sc, vw, len(views), rv[idx].copy(), ru[idx].copy(), rr[idx].copy(), nthreads)
    del keep
    return dict(image=img, flags=flags, nsamples=ns, neval=ne, ties=dict(index=idx, cand=cand, ncand=ncand))


def match_error(got, ref):
    """Per-pixel error of ``got`` ([..., 4], same layout as ref["image"]) against
    the oracle: the largest channel difference from the oracle image, or, for a
    pixel with several valid images (FLAG_ERT), from the closest of them (inf
    when they were too many to list).  Returns an array shaped like ``flags``."""
    g = np.asarray(got, np.float64).reshape(-1, 4)
    err = np.abs(g - ref["image"].reshape(-1, 4)).max(axis=1)
    t = ref["ties"]
    if t["index"].size:
        gi = g[t["index"]][:, None, :]
        e = np.abs(gi - t["cand"]).max(axis=2)  # [n][MAXC]
        valid = np.arange(MAXC)[None, :] < t["ncand"][:, None]
        best = np.where(valid, e, np.inf).min(axis=1)
        err[t["index"]] = best
    return err.reshape(ref["flags"].shape)


def render_grad(vol, tf, view, W, H, grad_out, vmin, vmax, step=0.5, tau=2.0, extent=0.0,
                want_vol=True, nthreads=0, eye_dist=0.0):
    """Exact FP64 gradient of sum(grad_out * image) w.r.t. the TF table and the voxels.

    Returns (grad_tf [M][4], grad_vol [n3][n2][n1] or None, image [H][W][4]).
    """
    sc, keep = _scene(vol, tf, vmin, vmax, step, tau, None, 0.0, 0.0)
    vw = _views([view], W, H, extent, eye_dist)
    g = np.ascontiguousarray(grad_out, np.float64).reshape(H, W, 4)
    M = sc.M
    gtf = np.zeros((M, 4), np.float64)
    gvol = np.zeros(np.asarray(vol).shape, np.float64) if want_vol else None
    img = np.zeros((H, W, 4), np.float64)
    rc = lib().or_render_grad(C.byref(sc), vw, _ptr(g), _ptr(gtf), _ptr(gvol), _ptr(img),
                              int(nthreads))
    if rc != 0:
        raise ValueError("oracle render_grad: bad input")
    del keep
    return gtf, gvol, img


def minmax(x, nthreads=0):
    """Global (min, max) in float64 and the count of non-finite values."""
    x = np.ascontiguousarray(x, np.float32)
    mn, mx, bad = C.c_double(), C.c_double(), C.c_int64()
    lib().or_minmax(_ptr(x), x.size, C.byref(mn), C.byref(mx), C.byref(bad), int(nthreads))
    return mn.value, mx.value, bad.value


def box_minmax(vol, lo, hi):
    """(min, max) over the inclusive voxel range [lo, hi] (axis order 1, 2, 3)."""
    vol = np.ascontiguousarray(vol, np.float32)
    n = np.array([vol.shape[2], vol.shape[1], vol.shape[0]], np.int64)
    lo = np.asarray(lo, np.int64)
    hi = np.asarray(hi, np.int64)
    mn, mx = C.c_double(), C.c_double()
    lib().or_box_minmax(_ptr(vol), _ptr(n), _ptr(lo), _ptr(hi), C.byref(mn), C.byref(mx))
    return mn.value, mx.value


def composite(layers):
    """Over-composite premultiplied RGBA layers [n][..., 4], front first."""
    L = np.ascontiguousarray(layers, np.float64)
    n = L.shape[0]
    npix = L[0].size // 4
    out = np.zeros(L.shape[1:], np.float64)
    lib().or_composite(_ptr(L), n, npix, _ptr(out))
    return out


def stored_box(lo, hi, dims, ghost=1):
    """Voxel range a sub-volume reads (its ownership box plus a ghost layer)."""
    slo = [max(0, int(lo[i]) - ghost) for i in range(3)]
    shi = [min(dims[i] - 1, int(hi[i]) + ghost) for i in range(3)]
    return slo, shi
