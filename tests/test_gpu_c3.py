"""The 2048 x 2048 x 1536 (24 GiB) workload at full size, in the launch
configuration the benchmark times (256^3 bricks, 16^3 macrocells, the permuted
copy, 1024^2 frames), against the FP64 oracle on sampled rays:

* the benchmark's four views that include the two looking along axis 1
  (rendered from the copy), ramp table, per-brick termination;
* perspective frames, whole-ray termination and MIP of the same views;
* a channel mask that switches off a band of spectral channels.

Rays: every 32nd row and column of each frame (1024 rays per frame) plus the
frame's centre row.
"""
import numpy as np
import pytest

import oracle
import paper_1008_0135_amd as vr
import synth
from gpu_util import parity

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

C = synth.CONFIGS["C3"]
DIMS = C["dims"]
W, H = C["image"]


def _say(msg):
    print(f"[gpu] {msg}", flush=True)


@pytest.fixture(scope="module")
def scene():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    _say("C3: generating the 24 GiB cube")
    vol = synth.config_cube("C3")
    ctx = vr.vr_create(0)
    h = vr.vr_volume_create(ctx, vol, DIMS, on_device=False)
    mn, mx = vr.vr_volume_minmax(h)
    vr.vr_volume_brick(h, vr.grid_spec(C["bricks"], macrocell=16, twin=True))
    views = synth.random_views(C["nviews"], C["view_seed"])
    # views 1 and 8 look mostly along axis 1 (rendered from the permuted copy)
    pick = [0, 1, 8, 12]
    assert all(abs(views[i][2][0]) > max(abs(views[i][2][1]), abs(views[i][2][2])) for i in (1, 8))
    yield dict(vol=vol, ctx=ctx, h=h, mn=mn, mx=mx, views=[views[i] for i in pick])
    vr.vr_volume_destroy(h)
    vr.vr_destroy(ctx)


def _rays(nv):
    yy, xx = np.meshgrid(np.arange(7, H, 32), np.arange(11, W, 32), indexing="ij")
    cy = np.full(W // 8, H // 2)
    cx = np.arange(0, W, 8)
    y = np.concatenate([yy.ravel(), cy])
    x = np.concatenate([xx.ravel(), cx])
    vv = np.repeat(np.arange(nv), y.size)
    return vv, np.tile(x, nv), np.tile(y, nv)


def _check(sc, tf, params, label, eye=0.0, mode=0, bricks=True, mask=None, window=None, lit=0):
    ctx, h, views = sc["ctx"], sc["h"], sc["views"]
    mn, mx = window if window else (sc["mn"], sc["mx"])
    vr.vr_tf_set(ctx, tf, mn, mx)
    vr.vr_mask_set(ctx, mask)
    out = torch.empty((len(views), H, W, 4), device="cuda")
    vr.vr_render(ctx, h, [vr.make_view(R, W, H, eye_dist=eye) for R in views], params, out)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    vr.vr_mask_set(ctx, None)
    vv, xx, yy = _rays(len(views))
    if lit:
        # also the pixels under the brightest compact sources (a table that is
        # transparent below several sigma leaves few strided rays lit): source
        # centres from the generator, projected with the orthographic camera
        srcs = sorted(synth.config_sources("C3"), key=lambda t: -t[0])[:lit]
        cen = np.array([c for _, c, _ in srcs], np.float64)
        mid = (np.array(DIMS, np.float64) - 1) / 2
        S = float(np.sqrt(((np.array(DIMS, np.float64) - 1) ** 2).sum()))
        for v, R in enumerate(views):
            u = np.floor(((cen - mid) @ R[0] / S + 0.5) * W).astype(int)
            w = np.floor(((cen - mid) @ R[1] / (S * H / W) + 0.5) * H).astype(int)
            ok = (u >= 0) & (u < W) & (w >= 0) & (w < H)
            vv = np.concatenate([vv, np.full(int(ok.sum()), v)])
            xx = np.concatenate([xx, u[ok]])
            yy = np.concatenate([yy, w[ok]])
    _say(f"C3 {label}: oracle on {vv.size} rays")
    ref = oracle.render_rays(sc["vol"], tf, views, W, H, vv, xx, yy, mn, mx, tau=0.99, mode=mode, eye_dist=eye,
                             bricks={"grid": C["bricks"]} if bricks else None, mask=mask)
    s = parity(got[vv, yy, xx], ref, label=f"C3 {label}")
    if lit:
        s["lit"] = int((ref["image"][:, 3] > 0).sum())
        assert s["lit"] >= 200, s
    _say(f"  {s}")
    assert np.isfinite(got).all() and (got >= 0).all() and (got <= 1.0 + 1e-6).all()


def test_c3_benchmark_views(scene):
    _check(scene, synth.tf_ramp(256), vr.make_params(), "ramp, per-brick termination")


def test_c3_perspective_global_mip(scene):
    n = np.array(DIMS, np.float64)
    eye = float(np.sqrt(((n - 1) ** 2).sum()))  # as in the benchmark's perspective leg
    _check(scene, synth.tf_ramp(256), vr.make_params(), "perspective", eye=eye)
    tf = synth.tf_colour(256)
    tf[:, 3] = np.minimum(1.0, tf[:, 3] * 4)
    _check(scene, tf, vr.make_params(ert_scope=vr.VR_ERT_GLOBAL), "whole-ray termination", bricks=False)
    mn, mx = scene["mn"], scene["mx"]
    _check(scene, tf, vr.make_params(mode=vr.VR_MODE_MIP), "MIP", mode=oracle.MODE_MIP,
           window=(mn, mn + 0.4 * (mx - mn)))


def test_c3_noise_suppressing_table(scene):
    """The second benchmark table: opacity 0 below 6 sigma, 16^3 macrocells, no mask
    (the plain empty-space-skipping ring march)."""
    tf = synth.tf_noise_suppress(scene["mn"], scene["mx"], thresh=6.0)
    _check(scene, tf, vr.make_params(), "noise-suppressing table, macrocell skipping", lit=400)


def test_c3_channel_mask(scene):
    mask = np.ones(DIMS[2], np.float32)
    mask[600:900] = 0.0
    mask[900:940] = np.linspace(0, 1, 40, dtype=np.float32)
    tf = synth.tf_noise_suppress(scene["mn"], scene["mx"], thresh=4.0, amax=0.3)
    _check(scene, tf, vr.make_params(), "channel mask, noise-suppressing table (macrocells active)", mask=mask)
