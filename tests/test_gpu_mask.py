"""GPU checks of the spectral-channel mask (through the C ABI).

* parity with the FP64 oracle: unbricked, grid and longest-axis bricks, views
  rendered from the permuted copy, perspective, MIP, whole-ray termination,
  with a band of switched-off channels and with random weights;
* an all-ones mask gives the same bits as no mask; the ring and gather marches
  give the same bits under a mask;
* a mask of the wrong length is rejected; the adjoint and the batched launch
  refuse to run while a mask is set; removing the mask restores the image.
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
    vr.vr_mask_set(c, None)
    vr.vr_destroy(c)


def _render(ctx, h, views, W, H, params, eye=0.0):
    out = torch.full((len(views), H, W, 4), -7.0, device="cuda")
    vr.vr_render(ctx, h, [vr.make_view(R, W, H, eye_dist=eye) for R in views], params, out)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def _ctx_with_march(mode):
    import os
    env = {"VR_MARCH": "ring", "VR_RING_SLOTS": "2"} if mode == "ring2" else {"VR_MARCH": mode}
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


DIMS = (90, 84, 100)


def _masks(n3):
    band = np.ones(n3, np.float32)
    band[30:55] = 0.0
    rnd = np.random.Generator(np.random.PCG64(161)).uniform(0, 1, n3).astype(np.float32)
    return {"band": band, "random": rnd}


def _axis1_view(seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    while True:
        R = synth.random_rotation(rng)
        if abs(R[2][0]) > max(abs(R[2][1]), abs(R[2][2])):
            return R


@pytest.mark.parametrize("layout,eye,mode,scope", [("whole", 0.0, 0, 0), ("grid", 0.0, 0, 0), ("kd", 0.0, 0, 0),
                                                   ("twin", 0.0, 0, 0), ("grid", 120.0, 0, 0), ("kd", 0.0, 1, 0),
                                                   ("grid", 0.0, 0, 1)])
def test_mask_parity_with_oracle(ctx, layout, eye, mode, scope):
    _say(f"channel mask parity vs oracle {layout} eye {eye} mode {mode} scope {scope}")
    vol = synth.cube(*DIMS, seed=162, n_sources=8, sigma_range=(2.0, 4.0))
    h = vr.vr_volume_create(ctx, vol, DIMS)
    bricks = None
    if layout in ("grid", "twin"):
        vr.vr_volume_brick(h, vr.grid_spec((40, 36, 48), twin=layout == "twin"))
        bricks = {"grid": (40, 36, 48)}
    elif layout == "kd":
        vr.vr_volume_brick(h, vr.kd_spec(6))
        bricks = oracle.kd_boxes(DIMS, 6)
    mn, mx = float(vol.min()), float(vol.max())
    tf = synth.tf_colour(256)
    tf[:, 3] = np.minimum(1.0, tf[:, 3] * 6)
    vr.vr_tf_set(ctx, tf, mn, mx)
    views = synth.random_views(2, 163) + [_axis1_view(164)]
    for name, mask in _masks(DIMS[2]).items():
        vr.vr_mask_set(ctx, mask)
        img = _render(ctx, h, views, 112, 96, vr.make_params(tau=0.99, mode=mode, ert_scope=scope), eye)
        ref = oracle.render(vol, tf, views, 112, 96, mn, mx, tau=0.99, mode=mode, eye_dist=eye, mask=mask,
                            bricks=None if scope else bricks)
        _say(f"  {name}: {parity(img, ref, label=f'mask {name} {layout}')}")
    vr.vr_mask_set(ctx, None)
    vr.vr_volume_destroy(h)


def test_mask_bits_marches_and_errors():
    _say("channel mask: all-ones == none; ring / gather bit identity; errors")
    dims = (120, 100, 140)
    vol = synth.cube(*dims, seed=165, n_sources=10, sigma_range=(2.0, 4.0))
    mn, mx = float(vol.min()), float(vol.max())
    views = synth.random_views(4, 166)
    mask = _masks(dims[2])["band"]
    imgs = {}
    for march in ("gather", "auto", "ring2"):
        c = _ctx_with_march(march)
        vr.vr_tf_set(c, synth.tf_colour(256), mn, mx)
        h = vr.vr_volume_create(c, vol, dims)
        vr.vr_volume_brick(h, vr.grid_spec((48, 40, 56), macrocell=8))
        plain = _render(c, h, views, 144, 128, vr.make_params())
        vr.vr_mask_set(c, np.ones(dims[2], np.float32))
        assert np.array_equal(_render(c, h, views, 144, 128, vr.make_params()), plain)
        vr.vr_mask_set(c, torch.from_numpy(mask).cuda())
        imgs[march] = _render(c, h, views, 144, 128, vr.make_params())
        assert np.abs(imgs[march] - plain).max() > 1e-3
        vr.vr_mask_set(c, mask[:-1])  # the wrong length for this volume
        with pytest.raises(vr.VRError) as e:
            _render(c, h, views, 32, 32, vr.make_params())
        assert e.value.code == vr.VR_EINVAL
        vr.vr_mask_set(c, None)
        assert np.array_equal(_render(c, h, views, 144, 128, vr.make_params()), plain)
        vr.vr_volume_destroy(h)
        vr.vr_destroy(c)
    assert np.array_equal(imgs["gather"], imgs["auto"]) and np.array_equal(imgs["gather"], imgs["ring2"])
    c = vr.vr_create(0)
    for bad in (np.array([0.5, 1.5, 0.2], np.float32), np.array([0.5, np.nan, 0.2], np.float32)):
        with pytest.raises(vr.VRError) as e:
            vr.vr_mask_set(c, bad)
        assert e.value.code == vr.VR_EINVAL
    small = synth.cube(30, 28, 32, seed=167, n_sources=2, sigma_range=(1.5, 3.0))
    d = torch.from_numpy(small).cuda()
    h = vr.vr_volume_wrap(c, d, (30, 28, 32))
    vr.vr_tf_set(c, synth.tf_colour(32))
    vr.vr_mask_set(c, np.ones(32, np.float32))
    out = torch.empty((1, 16, 16, 4), device="cuda")
    with pytest.raises(vr.VRError) as e:
        vr.vr_render(c, h, [vr.make_view(np.eye(3), 16, 16)], vr.make_params(), out, save=True)
    assert e.value.code == vr.VR_EUNSUPPORTED
    req = vr.make_request(h, np.eye(3), 16, 16, torch.from_numpy(synth.tf_colour(32)).cuda(), 0.0, 0.0, out[0])
    with pytest.raises(vr.VRError) as e:
        vr.vr_render_batch(c, [req], vr.make_params())
    assert e.value.code == vr.VR_EUNSUPPORTED
    vr.vr_volume_destroy(h)
    vr.vr_destroy(c)
