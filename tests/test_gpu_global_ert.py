"""GPU checks of early termination over the whole ray (VR_ERT_GLOBAL).

* bricked renders (grid, longest-axis, materialised; orthographic and
  perspective) match the FP64 oracle's unbricked image, ties in the opacity
  test aside;
* the ring and gather marches give the same bits, and macrocell skipping
  changes no bit;
* without termination the global and the per-brick (sort-last) images agree
  to rounding;
* MIP ignores the scope; per-brick images are refused under it.
"""
import numpy as np
import pytest

import oracle
import paper_1008_0135_amd as vr
import synth
from gpu_util import parity

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

G = vr.VR_ERT_GLOBAL


def _say(msg):
    print(f"[gpu] {msg}", flush=True)


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = vr.vr_create(0)
    yield c
    vr.vr_destroy(c)


def _render(ctx, h, views, W, H, params, eye=0.0):
    out = torch.full((len(views), H, W, 4), -7.0, device="cuda")
    vr.vr_render(ctx, h, [vr.make_view(R, W, H, eye_dist=eye) for R in views], params, out)
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


def _opaque_tf():
    tf = synth.tf_colour(256)
    tf[:, 3] = np.minimum(1.0, tf[:, 3] * 12)  # rays cross tau = 0.99 inside the volume
    return tf


@pytest.mark.parametrize("layout,eye", [("grid", 0.0), ("kd", 0.0), ("mat", 0.0), ("grid", 110.0), ("kd", 150.0)])
def test_global_matches_unbricked_oracle(ctx, layout, eye):
    _say(f"global termination parity vs unbricked oracle {DIMS} {layout} eye {eye}")
    vol = synth.cube(*DIMS, seed=121, n_sources=10, sigma_range=(2.0, 4.0))
    h = vr.vr_volume_create(ctx, vol, DIMS)
    spec = {"grid": vr.grid_spec((32, 40, 28)), "kd": vr.kd_spec(9),
            "mat": vr.grid_spec((48, 27, 56), materialize=True)}[layout]
    vr.vr_volume_brick(h, spec)
    mn, mx = float(vol.min()), float(vol.max())
    tf = _opaque_tf()
    vr.vr_tf_set(ctx, tf, mn, mx)
    views = synth.random_views(3, 122)
    img = _render(ctx, h, views, 128, 112, vr.make_params(tau=0.99, ert_scope=G), eye)
    ref = oracle.render(vol, tf, views, 128, 112, mn, mx, tau=0.99, eye_dist=eye)
    assert (ref["image"][..., 3] >= 0.99).mean() > 0.2  # termination decides many rays
    s = parity(img, ref, label=f"global ERT {layout}")
    _say(f"  {s}")
    local = _render(ctx, h, views, 128, 112, vr.make_params(tau=0.99), eye)
    assert np.abs(local - img).max() > 1e-3  # the per-brick test gives another image
    vr.vr_volume_destroy(h)


def test_global_marches_identical_and_skipping_inert():
    _say("global termination: ring / gather bit identity; macrocell skipping inert")
    dims = (150, 120, 170)
    vol = synth.cube(*dims, seed=123, n_sources=14, sigma_range=(2.0, 4.0))
    mn, mx = float(vol.min()), float(vol.max())
    low = synth.tf_noise_suppress(mn, mx, thresh=3.0, amax=0.6)
    views = synth.random_views(4, 124)
    layouts = {"grid": vr.grid_spec((64, 48, 40), macrocell=8), "kd": vr.kd_spec(11, macrocell=12)}
    imgs = {}
    for march in ("gather", "auto"):
        c = _ctx_with_march(march)
        h = vr.vr_volume_create(c, vol, dims)
        for name, spec in layouts.items():
            vr.vr_volume_brick(h, spec)
            for tname, tf in (("opaque", _opaque_tf()), ("low", low)):
                vr.vr_tf_set(c, tf, mn, mx)
                for eye in (0.0, 160.0):
                    on = _render(c, h, views, 160, 136, vr.make_params(tau=0.99, ert_scope=G), eye)
                    off = _render(c, h, views, 160, 136, vr.make_params(tau=0.99, ert_scope=G, ess=0), eye)
                    assert np.array_equal(on, off), (march, name, tname, eye)
                    imgs[(march, name, tname, eye)] = on
        vr.vr_volume_destroy(h)
        vr.vr_destroy(c)
    for k in [k for k in imgs if k[0] == "gather"]:
        a, b = imgs[k], imgs[("auto",) + k[1:]]
        assert np.array_equal(a, b), (k, float(np.abs(a - b).max()))


def test_global_equals_local_without_termination(ctx):
    _say("global vs per-brick without termination")
    vol = synth.cube(*DIMS, seed=125, n_sources=6, sigma_range=(2.0, 4.0))
    h = vr.vr_volume_create(ctx, vol, DIMS)
    vr.vr_volume_brick(h, vr.grid_spec((32, 32, 32)))
    vr.vr_tf_set(ctx, synth.tf_colour(256))
    views = synth.random_views(3, 126)
    for eye in (0.0, 120.0):
        g = _render(ctx, h, views, 96, 80, vr.make_params(tau=2.0, ert_scope=G), eye)
        loc = _render(ctx, h, views, 96, 80, vr.make_params(tau=2.0), eye)
        assert np.abs(g - loc).max() <= 2e-6
        assert (g[..., 3] > 0.05).mean() > 0.3
    vr.vr_volume_destroy(h)


def test_global_scope_mip_and_brick_images(ctx):
    _say("global termination: MIP unaffected, per-brick images refused")
    vol = synth.cube(*DIMS, seed=127, n_sources=6, sigma_range=(2.0, 4.0))
    h = vr.vr_volume_create(ctx, vol, DIMS)
    vr.vr_volume_brick(h, vr.grid_spec((32, 32, 32)))
    vr.vr_tf_set(ctx, synth.tf_colour(64))
    views = synth.random_views(2, 128)
    a = _render(ctx, h, views, 96, 80, vr.make_params(mode=vr.VR_MODE_MIP, ert_scope=G))
    b = _render(ctx, h, views, 96, 80, vr.make_params(mode=vr.VR_MODE_MIP))
    assert np.array_equal(a, b)
    with pytest.raises(vr.VRError) as e:
        vr.vr_render_bricks(ctx, h, vr.make_view(views[0], 96, 80), vr.make_params(ert_scope=G))
    assert e.value.code == vr.VR_EUNSUPPORTED
    with pytest.raises(vr.VRError) as e:
        vr.vr_render(ctx, h, [vr.make_view(views[0], 96, 80)], vr.make_params(ert_scope=5),
                     torch.empty((1, 80, 96, 4), device="cuda"))
    assert e.value.code == vr.VR_EINVAL
    vr.vr_volume_destroy(h)
