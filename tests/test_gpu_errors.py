"""Failure handling through the C ABI (status codes and the context staying
usable afterwards):

* VR_ENOMEM: a volume larger than the device's free memory (the allocation
  fails before the source is read);
* VR_ESTATE: a render on a context with no transfer function; a backward
  after the table changed since its forward; a backward with another
  volume's state;
* after each failure the same context renders a small volume correctly.
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


def _small_render_ok(ctx):
    vol = synth.cube(24, 20, 28, seed=201, n_sources=3, sigma_range=(2.0, 3.0))
    h = vr.vr_volume_create(ctx, vol, (24, 20, 28))
    tf = synth.tf_colour(64)
    mn, mx = float(vol.min()), float(vol.max())
    vr.vr_tf_set(ctx, tf, mn, mx)
    R = synth.random_views(1, 202)[0]
    out = torch.empty((1, 30, 32, 4), device="cuda")
    vr.vr_render(ctx, h, [vr.make_view(R, 32, 30)], vr.make_params(tau=0.99), out)
    torch.cuda.synchronize()
    ref = oracle.render(vol, tf, [R], 32, 30, mn, mx, tau=0.99)
    parity(out.cpu().numpy(), ref, label="render after a failure")
    vr.vr_volume_destroy(h)


def test_volume_larger_than_free_memory():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ctx = vr.vr_create(0)
    try:
        free, total = torch.cuda.mem_get_info()
        n1 = n2 = 16384
        n3 = int((free + 8 * 2**30) // (4 * n1 * n2)) + 1  # 8 GiB more than is free
        _say(f"VR_ENOMEM: volume of {4 * n1 * n2 * n3 / 2**30:.0f} GiB with {free / 2**30:.0f} GiB free")
        dummy = np.zeros(16, np.float32)  # never read: the allocation fails first
        with pytest.raises(vr.VRError) as e:
            vr.vr_volume_create(ctx, dummy, (n1, n2, n3), on_device=False)
        assert e.value.code == vr.VR_ENOMEM
        _small_render_ok(ctx)
    finally:
        vr.vr_destroy(ctx)


def test_render_without_table_and_stale_backward():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ctx = vr.vr_create(0)
    try:
        vol = synth.cube(20, 18, 22, seed=203, n_sources=3, sigma_range=(2.0, 3.0))
        dvol = torch.from_numpy(vol).cuda()
        h = vr.vr_volume_wrap(ctx, dvol, (20, 18, 22))
        R = synth.random_views(1, 204)[0]
        view = vr.make_view(R, 24, 20)
        params = vr.make_params(tau=2.0)
        out = torch.empty((1, 20, 24, 4), device="cuda")
        _say("VR_ESTATE: render before any transfer function")
        with pytest.raises(vr.VRError) as e:
            vr.vr_render(ctx, h, [view], params, out)
        assert e.value.code == vr.VR_ESTATE
        tf = synth.tf_colour(32)
        mn, mx = float(vol.min()) - 0.5, float(vol.max()) + 0.5
        vr.vr_tf_set(ctx, tf, mn, mx)
        st = vr.vr_render(ctx, h, [view], params, out, save=True)
        g = torch.ones_like(out)
        gtf = torch.empty((32, 4), device="cuda")
        gvol = torch.empty_like(dvol)
        vr.vr_render_backward(ctx, h, st, g, gtf, gvol)  # the state matches: fine
        _say("VR_ESTATE: backward after the table changed")
        vr.vr_tf_set(ctx, synth.tf_ramp(32), mn, mx)
        with pytest.raises(vr.VRError) as e:
            vr.vr_render_backward(ctx, h, st, g, gtf, gvol)
        assert e.value.code == vr.VR_ESTATE
        _say("VR_ESTATE: backward with another volume's state")
        h2 = vr.vr_volume_wrap(ctx, dvol, (20, 18, 22))
        vr.vr_tf_set(ctx, tf, mn, mx)
        st2 = vr.vr_render(ctx, h2, [view], params, out, save=True)
        with pytest.raises(vr.VRError) as e:
            vr.vr_render_backward(ctx, h, st2, g, gtf, gvol)
        assert e.value.code == vr.VR_ESTATE
        vr.vr_state_destroy(st)
        vr.vr_state_destroy(st2)
        vr.vr_volume_destroy(h)
        vr.vr_volume_destroy(h2)
        torch.cuda.synchronize()
        _small_render_ok(ctx)
    finally:
        vr.vr_destroy(ctx)
