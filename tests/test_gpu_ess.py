"""GPU checks of macrocell empty-space skipping (through the C ABI).

* macrocell (min, max) grids equal a direct reduction over each macrocell's
  voxels (ragged edges, several runs of macrocells along axis 1, a volume
  smaller than one macrocell, a non-finite voxel);
* rendering with skipping on is bit-identical to skipping off, for tables
  whose zero-opacity entries sit at the bottom, in the middle or nowhere,
  across table changes (re-classification), grid and longest-axis bricks,
  virtual and materialised storage, with and without early termination, in
  the default (ring) march and in the LDS-slab march;
* parity of a skipped render with the FP64 oracle.
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


def _expected_mc(vol, e):
    n3, n2, n1 = vol.shape
    c = [-(-(n - 1) // e) for n in (n1, n2, n3)]
    out = np.empty((c[2], c[1], c[0], 2), np.float32)
    for m3 in range(c[2]):
        for m2 in range(c[1]):
            for m1 in range(c[0]):
                box = vol[m3 * e:min(m3 * e + e, n3 - 1) + 1, m2 * e:min(m2 * e + e, n2 - 1) + 1,
                          m1 * e:min(m1 * e + e, n1 - 1) + 1]
                if not np.isfinite(box).all():
                    out[m3, m2, m1] = (np.nan, np.nanmax(np.where(np.isfinite(box), box, np.nan)))
                else:
                    out[m3, m2, m1] = (box.min(), box.max())
    return tuple(c), out


def _check_mc(h, vol, e):
    edge, cnt, mm = vr.vr_volume_macrocell_info(h)
    c, ref = _expected_mc(vol, e)
    assert edge == e and cnt == c
    assert np.array_equal(np.isnan(mm[..., 0]), np.isnan(ref[..., 0]))
    ok = ~np.isnan(ref[..., 0])
    assert np.array_equal(mm[..., 0][ok], ref[..., 0][ok])
    assert np.array_equal(mm[..., 1], ref[..., 1])


@pytest.mark.parametrize("dims,e", [((70, 53, 41), 16), ((70, 53, 41), 7), ((70, 53, 41), 128),
                                    ((2100, 5, 4), 16), ((2100, 5, 4), 1024), ((33, 17, 9), 2)])
def test_macrocell_minmax(ctx, dims, e):
    _say(f"macrocell minmax dims={dims} edge={e}")
    n1, n2, n3 = dims
    vol = synth.cube(n1, n2, n3, seed=81, n_sources=3, sigma_range=(1.5, 3.0))
    h = vr.vr_volume_create(ctx, vol, dims)
    vr.vr_volume_brick(h, vr.grid_spec((32, 32, 32), macrocell=e))
    _check_mc(h, vol, e)
    vr.vr_volume_brick(h, vr.grid_spec((32, 32, 32)))  # re-bricking without macrocells drops them
    assert vr.vr_volume_macrocell_info(h)[0] == 0
    vr.vr_volume_destroy(h)


def test_macrocell_nonfinite_and_errors(ctx):
    _say("macrocell non-finite voxel (wrapped volume), invalid edges")
    vol = synth.cube(40, 30, 20, seed=82, n_sources=2, sigma_range=(1.5, 3.0))
    vol[7, 11, 21] = np.nan
    d = torch.from_numpy(vol).cuda()
    h = vr.vr_volume_wrap(ctx, d, (40, 30, 20))
    vr.vr_volume_brick(h, vr.kd_spec(3, macrocell=8))
    _check_mc(h, vol, 8)
    for bad in (1, -3, 1025):
        with pytest.raises(vr.VRError):
            vr.vr_volume_brick(h, vr.grid_spec((16, 16, 16), macrocell=bad))
    vr.vr_volume_destroy(h)


def _tables(vmin, vmax):
    """Zero opacity below 4 sigma; zero opacity in a middle band; none zero."""
    low = synth.tf_noise_suppress(vmin, vmax, thresh=4.0, amax=0.2)
    mid = synth.tf_colour(256)
    mid[60:200, 3] = 0.0
    full = synth.tf_colour(256)
    return {"low": low, "mid": mid, "full": full}


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


@pytest.mark.parametrize("spec_name,march", [("grid", "auto"), ("grid_mat", "auto"), ("kd", "auto"),
                                             ("grid", "slab"), ("kd", "slab")])
def test_skip_bit_identical(ctx, spec_name, march):
    n1, n2, n3 = 150, 120, 170
    _say(f"skip on/off bit identity {n1}x{n2}x{n3} {spec_name} march {march}")
    ctx = _ctx_with_march(march)
    vol = synth.cube(n1, n2, n3, seed=83, n_sources=10, sigma_range=(2.0, 4.0))
    h = vr.vr_volume_create(ctx, vol, (n1, n2, n3))
    spec = {"grid": vr.grid_spec((64, 64, 64), macrocell=8),
            "grid_mat": vr.grid_spec((75, 60, 85), materialize=True, macrocell=16),
            "kd": vr.kd_spec(5, macrocell=12)}[spec_name]
    vr.vr_volume_brick(h, spec)
    mn, mx = float(vol.min()), float(vol.max())
    views = synth.random_views(4, 84)
    for name, tf in _tables(mn, mx).items():
        vr.vr_tf_set(ctx, tf, mn, mx)
        for tau in (0.99, 2.0):
            on = _render(ctx, h, views, 160, 136, vr.make_params(tau=tau, ess=1))
            off = _render(ctx, h, views, 160, 136, vr.make_params(tau=tau, ess=0))
            assert np.array_equal(on, off), (spec_name, name, tau, float(np.abs(on - off).max()))
    vr.vr_volume_destroy(h)
    vr.vr_destroy(ctx)


def test_skip_parity_with_oracle(ctx):
    n1, n2, n3 = 96, 80, 112
    _say(f"skip parity vs oracle {n1}x{n2}x{n3}")
    vol = synth.cube(n1, n2, n3, seed=85, n_sources=6, sigma_range=(2.0, 4.0))
    h = vr.vr_volume_create(ctx, vol, (n1, n2, n3))
    vr.vr_volume_brick(h, vr.grid_spec((48, 40, 56), macrocell=8))
    mn, mx = float(vol.min()), float(vol.max())
    tf = synth.tf_noise_suppress(mn, mx, thresh=4.0, amax=0.2)
    # share of macrocells the table makes transparent (the skip has work to do)
    _, _, mm = vr.vr_volume_macrocell_info(h)
    u = (mm[..., 1].astype(np.float64) - mn) / (mx - mn) * 255.0
    hi = np.minimum(255, np.ceil(u).astype(int) + 1)
    zero_run = np.argmax(tf[:, 3] > 0)  # entries [0, zero_run) have opacity 0
    assert (hi < zero_run).mean() > 0.5
    vr.vr_tf_set(ctx, tf, mn, mx)
    views = synth.random_views(2, 86)
    img = _render(ctx, h, views, 128, 128, vr.make_params(tau=0.99, ess=1))
    ref = oracle.render(vol, tf, views, 128, 128, mn, mx, tau=0.99, bricks={"grid": (48, 40, 56)})
    parity(img, ref, label="macrocell skip")
    vr.vr_volume_destroy(h)
