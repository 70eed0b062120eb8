"""GPU checks of perspective projection (through the C ABI).

* parity with the FP64 oracle for an unbricked volume, grid bricks and
  longest-axis bricks, near and far eyes, with early termination, and for
  maximum intensity projection;
* the footprint-cell march (cells sized per brick), the ring march's 8 x 8
  tiles (one launch per view, or per class of bricks with similar windows) and
  the gather march give the same image bits (emission-absorption and MIP,
  virtual and materialised bricks), and macrocell skipping changes no bit;
* the batched launch gives the same bits as plain renders;
* table and voxel gradients vs the oracle's exact FP64 gradient;
* an eye inside the box's circumsphere is rejected.
"""
import numpy as np
import pytest

import oracle
import paper_1008_0135_amd as vr
import synth
from gpu_util import parity

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu] {msg}", flush=True)


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = vr.vr_create(0)
    yield c
    vr.vr_destroy(c)


def _render(ctx, h, views, W, H, params, eye):
    out = torch.full((len(views), H, W, 4), -7.0, device="cuda")
    vr.vr_render(ctx, h, [vr.make_view(R, W, H, eye_dist=eye) for R in views], params, out)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def _ctx_with_march(mode):
    """A context with one march forced; "auto:K": the default march (footprint
    cells sized per brick where every brick of the view suits them, else the
    ring march's 8 x 8 tiles) with the bricks launched in K classes of similar
    window size (K = 1: one launch per view); "tiles" / "tiles:K": the same
    with 8 x 8 tiles for every perspective view; "ovf": cells of about 64
    pixels not shrunk to 64 at most (the overflow gather kernel takes the
    rest)."""
    import os
    env = {"VR_MARCH": mode}
    if mode.startswith("auto:"):
        env = {"VR_MARCH": "auto", "VR_PERSP_CLASSES": mode[5:]}
    elif mode.startswith("tiles"):
        env = {"VR_MARCH": "auto", "VR_PERSP_CELLS": "0", "VR_PERSP_CLASSES": mode[6:] or "3"}
    elif mode == "ovf":  # cells of about 64 pixels, not shrunk: many pass their 64th pixel to the gather kernel
        env = {"VR_MARCH": "auto", "VR_FOOT_RAYS": "64", "VR_FOOT_MAXPX": "4096"}
    old = {k: os.environ.get(k) for k in env}
    os.environ.update(env)
    try:
        return vr.vr_create(0)
    finally:
        for k, v in old.items():
            if v is None:
                del os.environ[k]
            else:
                os.environ[k] = v


DIMS = (96, 80, 112)  # half diagonal 84.9


@pytest.mark.parametrize("layout,eye,mode", [("whole", 95.0, 0), ("grid", 95.0, 0), ("kd", 95.0, 0),
                                             ("grid", 300.0, 0), ("kd", 140.0, 1), ("whole", 120.0, 1)])
def test_persp_parity_with_oracle(ctx, layout, eye, mode):
    _say(f"perspective parity vs oracle {DIMS} {layout} eye {eye} mode {mode}")
    vol = synth.cube(*DIMS, seed=101, n_sources=8, sigma_range=(2.0, 4.0))
    h = vr.vr_volume_create(ctx, vol, DIMS)
    bricks = None
    if layout == "grid":
        vr.vr_volume_brick(h, vr.grid_spec((48, 40, 56)))
        bricks = {"grid": (48, 40, 56)}
    elif layout == "kd":
        vr.vr_volume_brick(h, vr.kd_spec(5))
        bricks = oracle.kd_boxes(DIMS, 5)
    mn, mx = float(vol.min()), float(vol.max())
    tf = synth.tf_colour(256)
    tf[:, 3] = np.minimum(1.0, tf[:, 3] * 4)
    vr.vr_tf_set(ctx, tf, mn, mx - (1.5 if mode else 0.0))
    views = synth.random_views(3, 102)
    img = _render(ctx, h, views, 128, 112, vr.make_params(tau=0.99, mode=mode), eye)
    ref = oracle.render(vol, tf, views, 128, 112, mn, mx - (1.5 if mode else 0.0), tau=0.99, bricks=bricks,
                        mode=mode, eye_dist=eye)
    s = parity(img, ref, label=f"perspective {layout}")
    _say(f"  {s}")
    vr.vr_volume_destroy(h)


def test_persp_marches_identical_and_skipping_inert():
    _say("perspective: footprint cells / ring tiles (one launch, or bricks in classes of similar window) / gather bit identity; macrocell skipping inert")
    dims = (150, 120, 170)
    vol = synth.cube(*dims, seed=103, n_sources=10, sigma_range=(2.0, 4.0))
    mn, mx = float(vol.min()), float(vol.max())
    tables = {"colour": synth.tf_colour(256), "low": synth.tf_noise_suppress(mn, mx, thresh=4.0, amax=0.2)}
    views = synth.random_views(4, 104) + [synth.rot_axis(2, 90.0)]
    layouts = {"whole": None, "grid": vr.grid_spec((64, 64, 64), macrocell=8), "kd": vr.kd_spec(7, macrocell=12),
               "mat": vr.grid_spec((75, 60, 85), materialize=True, macrocell=16)}
    imgs = {}
    for march in ("gather", "auto", "auto:1", "tiles", "tiles:1", "ovf"):
        c = _ctx_with_march(march)
        h = vr.vr_volume_create(c, vol, dims)
        for name, spec in layouts.items():
            if spec is not None:
                vr.vr_volume_brick(h, spec)
            for tname, tf in tables.items():
                vr.vr_tf_set(c, tf, mn, mx)
                for eye in (135.0, 400.0):
                    for mode in (0, 1):
                        p = vr.make_params(tau=0.99, mode=mode)
                        imgs[(march, name, tname, eye, mode)] = _render(c, h, views, 160, 136, p, eye)
                    if name != "whole":
                        off = _render(c, h, views, 160, 136, vr.make_params(tau=0.99, ess=0), eye)
                        assert np.array_equal(off, imgs[(march, name, tname, eye, 0)]), (march, name, tname, eye)
        vr.vr_volume_destroy(h)
        vr.vr_destroy(c)
    for k in [k for k in imgs if k[0] == "gather"]:
        for m in ("auto", "auto:1", "tiles", "tiles:1", "ovf"):
            a, b = imgs[k], imgs[(m,) + k[1:]]
            assert np.array_equal(a, b), (m, k, float(np.abs(a - b).max()))
    ref = oracle.render(vol, tables["colour"], views, 160, 136, mn, mx, tau=0.99, bricks={"grid": (64, 64, 64)},
                        eye_dist=135.0)
    parity(imgs[("auto", "grid", "colour", 135.0, 0)], ref, label="perspective ring march")


def test_persp_batch_matches_plain(ctx):
    _say("perspective: batched launch == plain renders")
    descs = synth.batch_requests(seed=105, nreq=8, dim_range=(24, 72), img_range=(16, 80))
    reqs, outs, plains = [], [], []
    vols = []
    for j, d in enumerate(descs):
        n1, n2, n3 = d["dims"]
        a = synth.cube(n1, n2, n3, seed=d["seed"], n_sources=d["n_sources"], sigma_range=(1.5, 3.0))
        h = vr.vr_volume_create(ctx, a, (n1, n2, n3))
        vols.append(h)
        half = 0.5 * float(np.sqrt((n1 - 1) ** 2 + (n2 - 1) ** 2 + (n3 - 1) ** 2))
        eye = half * (1.05 + 0.3 * j)
        tf = d["tf"]
        tft = torch.from_numpy(tf).cuda()
        W, H = d["image"]
        out = torch.zeros((H, W, 4), device="cuda")
        reqs.append(vr.make_request(h, d["view"], W, H, tft, 0.0, 0.0, out, eye_dist=eye))
        outs.append((out, tft))
        vr.vr_tf_set(ctx, tf)
        pl = torch.empty((1, H, W, 4), device="cuda")
        vr.vr_render(ctx, h, [vr.make_view(d["view"], W, H, eye_dist=eye)], vr.make_params(), pl)
        plains.append(pl)
    cache = vr.vr_render_batch(ctx, reqs, vr.make_params())
    torch.cuda.synchronize()
    for (out, _), pl in zip(outs, plains):
        assert np.array_equal(out.cpu().numpy(), pl[0].cpu().numpy())
    vr.vr_batch_destroy(cache)
    for h in vols:
        vr.vr_volume_destroy(h)


def test_persp_gradients_match_oracle(ctx):
    _say("perspective: adjoint vs FP64 oracle")
    dims = (48, 40, 56)
    vol = synth.cube(*dims, seed=106, n_sources=4, sigma_range=(2.0, 4.0))
    tf = synth.tf_colour(64)
    tf[:, 3] = np.minimum(1.0, tf[:, 3] * 3.0)
    vmin, vmax = float(vol.min()) - 0.5, float(vol.max()) + 0.5
    views = synth.random_views(2, 107)
    W = H = 64
    eye = 60.0  # half diagonal 42.4
    rng = np.random.Generator(np.random.PCG64(108))
    gout = rng.normal(0, 1, (2, H, W, 4))
    dvol = torch.from_numpy(vol).cuda()
    h = vr.vr_volume_wrap(ctx, dvol, dims)
    vr.vr_tf_set(ctx, tf, vmin, vmax)
    out = torch.empty((2, H, W, 4), device="cuda")
    vv = [vr.make_view(R, W, H, eye_dist=eye) for R in views]
    st = vr.vr_render(ctx, h, vv, vr.make_params(tau=2.0, ess=0), out, save=True)
    g = torch.from_numpy(np.ascontiguousarray(gout, np.float32)).cuda()
    gtf = torch.empty((tf.shape[0], 4), device="cuda")
    gvol = torch.empty_like(dvol)
    vr.vr_render_backward(ctx, h, st, g, gtf, gvol)
    torch.cuda.synchronize()
    otf = np.zeros((tf.shape[0], 4))
    ovol = np.zeros(vol.shape)
    for j, R in enumerate(views):
        a, b, img = oracle.render_grad(vol, tf, R, W, H, gout[j], vmin, vmax, tau=2.0, eye_dist=eye)
        otf += a
        ovol += b
        assert np.abs(out[j].cpu().numpy() - img).max() <= 2e-5
    for got, ref, name in ((gtf.cpu().numpy().astype(np.float64), otf, "tf"),
                           (gvol.cpu().numpy().astype(np.float64), ovol, "voxels")):
        scale = max(1e-3 * float(np.abs(ref).max()), 1e-30)
        rel = np.abs(got - ref) / np.maximum(np.abs(ref), scale)
        _say(f"  max rel err {name}: {rel.max():.3g}")
        assert rel.max() <= 1e-3
    vr.vr_state_destroy(st)
    vr.vr_volume_destroy(h)


def test_persp_eye_inside_rejected(ctx):
    vol = synth.cube(40, 36, 48, seed=109, n_sources=2, sigma_range=(1.5, 3.0))
    h = vr.vr_volume_create(ctx, vol, (40, 36, 48))
    vr.vr_tf_set(ctx, synth.tf_ramp(16))
    out = torch.empty((1, 16, 16, 4), device="cuda")
    with pytest.raises(vr.VRError) as e:
        vr.vr_render(ctx, h, [vr.make_view(np.eye(3), 16, 16, eye_dist=30.0)], vr.make_params(), out)
    assert e.value.code == vr.VR_EINVAL
    vr.vr_volume_destroy(h)
