"""GPU checks of maximum intensity projection (through the C ABI).

* parity with the FP64 oracle for an unbricked volume, grid bricks and
  longest-axis bricks, with a window that saturates some rays (so the stop at
  M = 1 is taken);
* the ring and gather marches give the same image bits, for every layout;
* tau, empty-space skipping and macrocells change nothing, and bricked images
  agree with the whole-volume image;
* the adjoint and the batched launch reject the mode.
"""
import numpy as np
import pytest

import oracle
import paper_1008_0135_amd as vr
import synth
from gpu_util import parity

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

MIP = vr.VR_MODE_MIP


def _say(msg):
    print(f"[gpu] {msg}", flush=True)


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = vr.vr_create(0)
    yield c
    vr.vr_destroy(c)


def _render(ctx, h, views, W, H, params):
    out = torch.full((len(views), H, W, 4), -7.0, device="cuda")
    vr.vr_render(ctx, h, [vr.make_view(R, W, H) for R in views], params, out)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def _ctx_with_march(mode):
    import os
    old = os.environ.get("VR_MARCH")
    os.environ["VR_MARCH"] = mode
    try:
        return vr.vr_create(0)
    finally:
        if old is None:
            del os.environ["VR_MARCH"]
        else:
            os.environ["VR_MARCH"] = old


DIMS = (96, 80, 112)
LAYOUTS = {"whole": None, "grid": (48, 40, 56), "kd": 5}


def _spec(name, macrocell=0):
    v = LAYOUTS[name]
    if v is None:
        return None
    if name == "kd":
        return vr.kd_spec(v, macrocell=macrocell)
    return vr.grid_spec(v, macrocell=macrocell)


def _oracle_bricks(name):
    v = LAYOUTS[name]
    if v is None:
        return None
    if name == "kd":
        return oracle.kd_boxes(DIMS, v)
    return {"grid": v}


@pytest.mark.parametrize("layout", list(LAYOUTS))
def test_mip_parity_with_oracle(ctx, layout):
    _say(f"MIP parity vs oracle {DIMS} {layout}")
    vol = synth.cube(*DIMS, seed=91, n_sources=8, sigma_range=(2.0, 4.0))
    h = vr.vr_volume_create(ctx, vol, DIMS)
    spec = _spec(layout)
    if spec is not None:
        vr.vr_volume_brick(h, spec)
    mn, mx = float(vol.min()), float(vol.max()) - 1.5  # rays through the peaks saturate
    tf = synth.tf_ramp(64)
    vr.vr_tf_set(ctx, tf, mn, mx)
    views = synth.random_views(3, 92)
    img = _render(ctx, h, views, 128, 112, vr.make_params(tau=0.99, mode=MIP))
    ref = oracle.render(vol, tf, views, 128, 112, mn, mx, tau=0.99, bricks=_oracle_bricks(layout),
                        mode=oracle.MODE_MIP)
    s = parity(img, ref, label=f"MIP {layout}")
    _say(f"  {s}")
    assert (img[..., 0] == 1.0).any() and ((img[..., 0] > 0) & (img[..., 0] < 1.0)).any()
    assert np.array_equal(img[..., 0], img[..., 3]) and np.array_equal(img[..., 1], img[..., 2])
    vr.vr_volume_destroy(h)


def test_mip_marches_identical_and_options_inert():
    _say("MIP: ring / gather bit identity; tau, skipping and macrocells inert")
    dims = (150, 120, 170)
    vol = synth.cube(*dims, seed=93, n_sources=10, sigma_range=(2.0, 4.0))
    mn, mx = float(vol.min()), float(vol.max())
    low = synth.tf_noise_suppress(mn, mx, thresh=4.0, amax=0.2)  # table with a long zero run
    views = synth.random_views(4, 94) + [synth.rot_axis(2, 90.0)]
    layouts = {"grid": vr.grid_spec((64, 64, 64), macrocell=8), "kd": vr.kd_spec(7, macrocell=12),
               "mat": vr.grid_spec((75, 60, 85), materialize=True)}
    imgs = {}
    for march in ("gather", "auto"):
        c = _ctx_with_march(march)
        vr.vr_tf_set(c, low, mn, mx - 2.0)
        h = vr.vr_volume_create(c, vol, dims)
        whole = _render(c, h, views, 160, 136, vr.make_params(mode=MIP))
        imgs[(march, "whole")] = whole
        for name, spec in layouts.items():
            vr.vr_volume_brick(h, spec)
            for W in (160, 333):
                imgs[(march, name, W)] = _render(c, h, views, W, W - 24, vr.make_params(tau=0.99, mode=MIP))
            alt = _render(c, h, views, 160, 136, vr.make_params(tau=0.3, ess=0, mode=MIP))
            assert np.array_equal(alt, imgs[(march, name, 160)]), (march, name)
            # the maximum needs no order: bricked images agree with the whole-volume
            # image up to the rounding of brick-local sample positions
            np.testing.assert_allclose(imgs[(march, name, 160)], whole, rtol=0, atol=2e-5)
        vr.vr_volume_destroy(h)
        vr.vr_destroy(c)
    for k in [k for k in imgs if k[0] == "gather"]:
        a, b = imgs[k], imgs[("auto",) + k[1:]]
        assert np.array_equal(a, b), (k, float(np.abs(a - b).max()))


def test_mip_unsupported_paths(ctx):
    _say("MIP: adjoint and batch reject the mode")
    vol = synth.cube(40, 36, 44, seed=95, n_sources=3, sigma_range=(1.5, 3.0))
    h = vr.vr_volume_create(ctx, vol, (40, 36, 44))
    tf = synth.tf_ramp(32)
    mn, mx = float(vol.min()), float(vol.max())
    vr.vr_tf_set(ctx, tf, mn, mx)
    out = torch.empty((1, 32, 32, 4), device="cuda")
    views = [vr.make_view(synth.random_views(1, 96)[0], 32, 32)]
    with pytest.raises(vr.VRError) as e:
        vr.vr_render(ctx, h, views, vr.make_params(mode=MIP), out, save=True)
    assert e.value.code == vr.VR_EUNSUPPORTED
    tft = torch.from_numpy(tf).cuda()
    req = vr.make_request(h, synth.random_views(1, 97)[0], 32, 32, tft, mn, mx, out)
    with pytest.raises(vr.VRError) as e:
        vr.vr_render_batch(ctx, [req], vr.make_params(mode=MIP))
    assert e.value.code == vr.VR_EUNSUPPORTED
    with pytest.raises(vr.VRError) as e:
        vr.vr_render(ctx, h, views, vr.make_params(mode=7), out)
    assert e.value.code == vr.VR_EINVAL
    vr.vr_volume_destroy(h)
