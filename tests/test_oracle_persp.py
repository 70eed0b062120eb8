"""Pins of the oracle's perspective camera.

* exact-rational brute force (whole volume, grid and longest-axis sub-volumes,
  with and without early termination) on tiny inputs;
* the centre pixel of an odd-sized image sees the orthographic centre ray;
* isolated bright voxels land, in a maximum intensity projection, on the pixel
  the pinhole projection x D / (D + z) predicts (and not where an orthographic
  or sign-flipped projection would put them);
* a 180-degree roll about the view axis flips the image;
* sub-volumes without early termination give the whole-volume image;
* a distant eye tends to the orthographic image.
"""
import numpy as np
import pytest

import oracle
import synth
from oracle import exact


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def _case(seed, dims=(5, 4, 6), M=8, amax=0.3):
    rng = _rng(seed)
    n1, n2, n3 = dims
    vol = rng.normal(0, 1, (n3, n2, n1)).astype(np.float32)
    tf = rng.uniform(0, 1, (M, 4)).astype(np.float32)
    tf[:, 3] *= amax
    R = synth.random_rotation(rng)
    return vol, tf, R


@pytest.mark.parametrize("seed,tau,D,kind", [(51, 2.0, 4.0, None), (52, 0.7, 9.0, None), (53, 0.6, 5.0, "grid"),
                                             (54, 2.0, 6.5, "kd"), (55, 0.8, 4.5, "kd")])
def test_exact_rational(orc, seed, tau, D, kind):
    dims = (5, 4, 6) if kind is None else (6, 5, 7)
    vol, tf, R = _case(seed, dims=dims)
    vmin, vmax = float(vol.min()) + 0.2, float(vol.max()) - 0.2
    W, H, ext = 6, 5, 7.0
    boxes = bricks = None
    if kind == "grid":
        boxes, _ = orc.grid_boxes(dims, (2, 3, 4))
        bricks = {"grid": (2, 3, 4)}
    elif kind == "kd":
        boxes = bricks = orc.kd_boxes(dims, 3)
    res = orc.render(vol, tf, [R], W, H, vmin, vmax, tau=tau, extent=ext, bricks=bricks, eye_dist=D)
    want = np.array(exact.to_float(exact.render(vol.tolist(), tf.tolist(), R.tolist(), W, H, ext, vmin, vmax,
                                                tau=tau, boxes=boxes, eye_dist=D)))
    assert ((res["flags"][0] & orc.FLAG_GEOM) == 0).all()
    np.testing.assert_allclose(res["image"][0], want, rtol=0, atol=1e-12)
    assert (want[..., 3] > 0).sum() >= 10


@pytest.mark.parametrize("seed", [61, 62, 63])
def test_centre_pixel_is_the_orthographic_centre_ray(orc, seed):
    vol = synth.cube(21, 19, 23, seed=seed, n_sources=3, sigma_range=(1.5, 3.0))
    tf = synth.tf_colour(64)
    R = synth.random_views(1, seed)[0]
    mn, mx = float(vol.min()), float(vol.max())
    ortho = orc.render(vol, tf, [R], 7, 5, mn, mx, tau=0.95)["image"][0]
    for D in (20.0, 35.0, 300.0):
        persp = orc.render(vol, tf, [R], 7, 5, mn, mx, tau=0.95, eye_dist=D)["image"][0]
        np.testing.assert_allclose(persp[2, 3], ortho[2, 3], rtol=0, atol=1e-12)
        assert not np.allclose(persp, ortho, atol=1e-6)  # off-centre rays do differ


def test_bright_voxels_land_on_the_pinhole_projection(orc):
    n = 41
    vol = np.zeros((n, n, n), np.float32)
    rng = _rng(71)
    pts = []
    while len(pts) < 6:
        q = rng.integers(6, n - 6, 3)
        if all(np.abs(q - p).max() > 8 for p in pts):
            pts.append(q)
    for q in pts:
        vol[q[2], q[1], q[0]] = 1.0
    R = synth.random_views(1, 72)[0]
    W = H = 160
    S = float(np.sqrt(3.0) * (n - 1))  # image width in voxels on the plane through the centre
    D = 45.0
    img = orc.render(vol, synth.tf_ramp(8), [R], W, H, 0.0, 1.0, tau=2.0, extent=S, eye_dist=D,
                     mode=oracle.MODE_MIP)["image"][0, ..., 0]
    c = np.full(3, (n - 1) / 2.0)
    shifts = []
    for q in pts:
        r = q - c
        x, y, z = r @ R[0], r @ R[1], r @ R[2]
        u = (x * D / (D + z) / S + 0.5) * W - 0.5
        v = (y * D / (D + z) / S + 0.5) * H - 0.5
        iu, iv = int(round(u)), int(round(v))
        win = img[iv - 3:iv + 4, iu - 3:iu + 4]
        jv, ju = np.unravel_index(np.argmax(win), win.shape)
        assert abs(iv - 3 + jv - v) <= 1.0 and abs(iu - 3 + ju - u) <= 1.0, (q, u, v)
        assert win.max() > 0.4
        # an orthographic projection would put the voxel this many pixels away
        shifts.append(np.hypot(x * (D / (D + z) - 1), y * (D / (D + z) - 1)) / S * W)
    assert max(shifts) > 4.0


def test_roll_180_flips(orc):
    vol = synth.cube(20, 18, 22, seed=81, n_sources=3, sigma_range=(1.5, 3.0))
    R = synth.random_views(1, 82)[0]
    Rroll = np.array([-R[0], -R[1], R[2]])
    tf = synth.tf_colour(32)
    mn, mx = float(vol.min()), float(vol.max())
    a = orc.render(vol, tf, [R], 16, 16, mn, mx, tau=0.9, eye_dist=30.0)
    b = orc.render(vol, tf, [Rroll], 16, 16, mn, mx, tau=0.9, eye_dist=30.0)
    np.testing.assert_allclose(a["image"][0], b["image"][0][::-1, ::-1], rtol=0, atol=1e-12)


@pytest.mark.parametrize("bricks", [{"grid": (8, 10, 12)}, "kd"])
def test_subvolumes_equal_whole_without_termination(orc, bricks):
    dims = (30, 26, 34)
    vol = synth.cube(*dims, seed=91, n_sources=4, sigma_range=(1.5, 3.0))
    if bricks == "kd":
        bricks = orc.kd_boxes(dims, 6)
    tf = synth.tf_colour(64)
    views = synth.random_views(3, 92)
    mn, mx = float(vol.min()), float(vol.max())
    whole = orc.render(vol, tf, views, 24, 20, mn, mx, tau=2.0, eye_dist=40.0)
    b = orc.render(vol, tf, views, 24, 20, mn, mx, tau=2.0, bricks=bricks, eye_dist=40.0)
    ok = (b["flags"] & orc.FLAG_GEOM) == 0
    np.testing.assert_allclose(b["image"][ok], whole["image"][ok], rtol=0, atol=1e-12)
    assert ok.mean() > 0.99


def test_distant_eye_tends_to_orthographic(orc):
    vol = synth.cube(24, 20, 28, seed=93, n_sources=3, sigma_range=(1.5, 3.0))
    tf = synth.tf_colour(64)
    views = synth.random_views(2, 94)
    mn, mx = float(vol.min()), float(vol.max())
    ortho = orc.render(vol, tf, views, 20, 20, mn, mx, tau=2.0)["image"]
    errs = []
    for D in (1e3, 1e5):
        p = orc.render(vol, tf, views, 20, 20, mn, mx, tau=2.0, eye_dist=D)["image"]
        errs.append(np.quantile(np.abs(p - ortho), 0.9))
    assert errs[1] < 1e-4 and errs[1] < errs[0]
