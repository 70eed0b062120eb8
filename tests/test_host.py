"""Host-side checks of libvr (no GPU needed).

* the shared library loads and exports every function include/vr.h declares;
* argument validation returns the documented status codes;
* the host-only planning helpers: partitions (vs the oracle's own partition
  code), rendering rectangles (contain every pixel whose ray meets the brick,
  checked by brute force over pixels), depth order (consistent with the
  per-ray order of brick entry points), nominal sample counts (vs the oracle).
"""
import ctypes as C
import math
import os
import re

import numpy as np
import pytest

import paper_1008_0135_amd as vr
import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "vr.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(vr_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    L = vr.lib()
    names = _declared()
    assert len(names) >= 25
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(vr.exported_symbols())
    assert vr.vr_version() == 2


def test_params_default():
    p = vr.make_params()
    assert p.step == 0.5 and p.tau == 0.99 and p.ess == 1 and p.ckpt_K == 32


def _rc(fn, *args):
    return fn(*args)


def test_error_paths_without_gpu():
    L = vr.lib()
    out = C.c_void_p()
    assert L.vr_create(0, None) == vr.VR_EINVAL
    assert L.vr_tf_set(None, None, 4, 0.0, 0.0, 0, 0) == vr.VR_EINVAL
    assert b"non-NULL" in L.vr_last_error()
    assert L.vr_volume_create(None, None, 0, 4, 4, 4, None, None, 0, C.byref(out)) == vr.VR_EINVAL
    assert L.vr_render(None, None, None, 1, None, None, 0, None) == vr.VR_EINVAL
    assert L.vr_composite(None, None, 0, None, 4, 4, None, 0) == vr.VR_EINVAL
    assert L.vr_render_backward(None, None, None, None, None, None, 0, 0) != vr.VR_OK
    for f in ("vr_destroy", "vr_volume_destroy", "vr_state_destroy", "vr_batch_destroy"):
        assert getattr(L, f)(None) == vr.VR_OK
    d = (C.c_int64 * 3)(1, 8, 8)
    v = vr.make_view(np.eye(3), 8, 8)
    n = C.c_int64()
    assert L.vr_count_samples(d, C.byref(v), 0.5, C.byref(n)) == vr.VR_EINVAL
    d = (C.c_int64 * 3)(8, 8, 8)
    assert L.vr_count_samples(d, C.byref(v), 0.0, C.byref(n)) == vr.VR_EINVAL
    bad = vr.make_view(np.zeros((3, 3)), 8, 8)
    assert L.vr_count_samples(d, C.byref(bad), 0.5, C.byref(n)) == vr.VR_EINVAL
    big = vr.make_view(np.eye(3), 20000, 8)
    assert L.vr_count_samples(d, C.byref(big), 0.5, C.byref(n)) == vr.VR_EINVAL
    spec = vr.grid_spec((0, 4, 4))
    nb = C.c_int32(0)
    assert L.vr_partition(d, C.byref(spec), C.byref(nb), None) == vr.VR_EINVAL
    spec = vr.kd_spec(0)
    assert L.vr_partition(d, C.byref(spec), C.byref(nb), None) == vr.VR_EINVAL


def test_create_without_gpu_reports_ehip():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(vr.VRError) as e:
        vr.vr_create(0)
    assert e.value.code == vr.VR_EHIP


def _boxes(descs):
    return [(tuple(d.lo), tuple(d.hi), tuple(d.closed)) for d in descs]


@pytest.mark.parametrize("dims,size", [((512, 512, 1024), (256, 256, 512)), ((2048, 2048, 1536), (256,) * 3),
                                       ((64, 40, 33), (16, 16, 16)), ((10, 11, 12), (3, 4, 5))])
def test_grid_partition_matches_oracle(orc, dims, size):
    got = _boxes(vr.vr_partition(dims, vr.grid_spec(size)))
    want, _ = orc.grid_boxes(dims, size)
    assert got == want


@pytest.mark.parametrize("dims,p", [((100, 60, 80), 3), ((512, 512, 1024), 8), ((33, 47, 29), 7), ((20, 20, 20), 5)])
def test_kd_partition_matches_oracle(orc, dims, p):
    got = _boxes(vr.vr_partition(dims, vr.kd_spec(p)))
    assert got == orc.kd_boxes(dims, p)


def test_stored_ranges_are_ghosted():
    descs = vr.vr_partition((64, 64, 64), vr.grid_spec((16, 16, 16)))
    d = descs[5]
    for i in range(3):
        assert d.slo[i] == max(0, d.lo[i] - 1)
        assert d.shi[i] == min(63, d.hi[i] + 1)


def _rays(dims, R, W, H, extent=0.0, eye_dist=0.0):
    n = np.array(dims, np.float64)
    c = (n - 1) / 2
    S = extent if extent > 0 else math.sqrt(((n - 1) ** 2).sum())
    u = np.arange(W)
    v = np.arange(H)
    x = ((u + 0.5) / W - 0.5) * S
    y = ((v + 0.5) / H - 0.5) * S * H / W
    R = np.asarray(R)
    if eye_dist > 0:
        w = x[None, :, None] * R[0] + y[:, None, None] * R[1] + eye_dist * R[2]
        d = w / np.linalg.norm(w, axis=-1, keepdims=True)
        o = np.broadcast_to(c - eye_dist * R[2], d.shape)
        return o, d
    o = c[None, None] + x[None, :, None] * R[0] + y[:, None, None] * R[1] - S * R[2]
    return o, R[2]


def _slab(o, d, lo, hi):
    with np.errstate(divide="ignore", invalid="ignore"):
        t1 = (lo - o) / d
        t2 = (hi - o) / d
    tn = np.where(d == 0, np.where((o >= lo) & (o <= hi), -np.inf, np.inf), np.minimum(t1, t2))
    tf = np.where(d == 0, np.where((o >= lo) & (o <= hi), np.inf, -np.inf), np.maximum(t1, t2))
    return tn.max(-1), tf.min(-1)


@pytest.mark.parametrize("kind,eye", [("grid", 0.0), ("kd", 0.0), ("grid", 90.0), ("kd", 90.0), ("grid", 260.0),
                                      ("kd", 260.0)])
def test_rectangles_conservative_and_order_consistent(kind, eye):
    """Rectangles hold every pixel whose ray meets the brick; the order and the
    waves sort every ray's bricks by entry (parallel rays, and rays from an eye
    at 90 or 260 voxels from the centre of a box of half-diagonal 86)."""
    dims = (96, 80, 120)
    spec = vr.grid_spec((32, 32, 48)) if kind == "grid" else vr.kd_spec(6)
    descs = vr.vr_partition(dims, spec)
    for R in synth.random_views(4, 41):
        W, H = 64, 48
        view = vr.make_view(R, W, H, eye_dist=eye)
        rects, order, waves = vr.vr_plan_view(dims, spec, view, waves=True)
        o, d = _rays(dims, R, W, H, eye_dist=eye)
        pos = {b: i for i, b in enumerate(order)}
        entries = []
        for b, dsc in enumerate(descs):
            lo = np.array(dsc.lo, np.float64)
            hi = np.array(dsc.hi, np.float64)
            tn, tf = _slab(o, d, lo, hi)
            hit = tn < tf
            x0, y0, w, h = rects[b]
            ys, xs = np.nonzero(hit)
            if len(xs):
                assert w > 0 and h > 0
                assert xs.min() >= x0 and xs.max() < x0 + w and ys.min() >= y0 and ys.max() < y0 + h
                # not wildly larger than needed (where the image does not cut the
                # projection: the box of a cut hull can exceed the visible part)
                if x0 > 0 and y0 > 0 and x0 + w < W and y0 + h < H:
                    assert x0 >= xs.min() - 3 and x0 + w <= xs.max() + 4
            entries.append(np.where(hit, tn, np.inf))
        E = np.stack(entries)  # [nb][H][W]
        # any two bricks a ray meets with distinct entries are ordered by entry
        for yy in range(0, H, 5):
            for xx in range(0, W, 5):
                met = [(E[b, yy, xx], b) for b in range(len(descs)) if np.isfinite(E[b, yy, xx])]
                met.sort()
                for (t1, b1), (t2, b2) in zip(met, met[1:]):
                    if t2 - t1 > 1e-9:
                        assert pos[b1] < pos[b2]
                        assert waves[b1] < waves[b2]  # global termination: one brick per ray per wave


def test_count_samples_matches_oracle(orc):
    dims = (40, 36, 48)
    vol = np.zeros((48, 36, 40), np.float32)
    tf = synth.tf_ramp(8)
    for R in synth.random_views(3, 42) + [np.eye(3)]:
        for eye in (0.0, 40.0, 150.0):
            view = vr.make_view(R, 64, 56, eye_dist=eye)
            n = vr.vr_count_samples(dims, view, 0.5)
            res = orc.render(vol, tf, [R], 64, 56, 0.0, 1.0, tau=2.0, eye_dist=eye)
            assert n == res["nsamples"]


def test_eye_distance_validation():
    dims = (40, 36, 48)  # half diagonal 35.19
    for bad in (-1.0, 20.0, 35.1, float("nan")):
        with pytest.raises(vr.VRError) as e:
            vr.vr_count_samples(dims, vr.make_view(np.eye(3), 16, 16, eye_dist=bad), 0.5)
        assert e.value.code == vr.VR_EINVAL
    vr.vr_count_samples(dims, vr.make_view(np.eye(3), 16, 16, eye_dist=35.3), 0.5)


def test_cell_traffic_model_terms_ordered():
    """The window-traffic model of the footprint-cell march (host only): the
    rendered bricks' own voxels are the cube's, each term adds a cost to the
    one before (lines of all windows >= 64-byte segments >= exact window bytes
    >= the line-granular union of the windows >= own voxels)."""
    dims = (512, 512, 384)
    spec = vr.grid_spec((128, 128, 128))
    for R in synth.random_views(5, 77) + [np.eye(3)]:
        t = vr.vr_plan_cells(dims, spec, vr.make_view(R, 256, 256))
        assert t.own_bytes == 4.0 * dims[0] * dims[1] * dims[2]
        assert t.own_bytes <= t.union_bytes <= t.window_bytes <= t.segment_bytes <= t.line_bytes
        assert 0 < t.rays_per_cell <= 64 and t.axis in (2, 3) and t.row_floats % 4 == 0 and t.rows > 0
        assert t.cells > 0 and t.cell_layers > t.cells
    # a permuted view is planned on the copy, with the copy's axes
    R1 = synth.rot_axis(2, 90.0)
    t = vr.vr_plan_cells(dims, vr.grid_spec((128, 128, 128), twin=True), vr.make_view(R1, 256, 256))
    assert t.twin == 1 and t.own_bytes == 4.0 * dims[0] * dims[1] * dims[2]
    with pytest.raises(vr.VRError):
        vr.vr_plan_cells(dims, spec, vr.make_view(np.eye(3), 256, 256, eye_dist=900.0))
    with pytest.raises(vr.VRError):
        vr.vr_plan_cells(dims, spec, vr.make_view(np.eye(3), 256, 256), rays=200.0)
