"""Pins of the oracle's maximum intensity projection (MIP).

* constant cube: every ray that meets the volume gives the normalised value;
* rays down voxel columns (identity view, one pixel per column): the maximum
  over the lattice of the linearly interpolated column, computed with numpy;
* the exact-rational brute force on tiny inputs, whole and in sub-volumes;
* sub-volumes (grid, longest-axis) give exactly the whole-volume image (the
  maximum needs no order), and early termination changes nothing;
* a 180-degree roll about the view axis flips the image.
"""
import numpy as np
import pytest

import oracle
import synth
from oracle import exact

MIP = oracle.MODE_MIP


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def test_constant_cube(orc):
    n = 12
    vol = np.full((n, n, n), 0.37, np.float32)
    tf = synth.tf_ramp(16)
    res = orc.render(vol, tf, [np.eye(3), synth.random_views(1, 3)[0]], 8, 8, 0.0, 1.0, tau=2.0,
                     extent=float(n - 1), mode=MIP)
    img = res["image"]
    hit = img[..., 3] > 0
    assert hit[0].all()  # the identity view covers the box face exactly
    np.testing.assert_allclose(img[hit], np.float32(0.37), rtol=0, atol=1e-12)
    assert (img[~hit] == 0).all()


def _column_mip(vol, vmin, vmax):
    n3 = vol.shape[0]
    nk = 2 * (n3 - 1)
    z = (np.arange(nk) + 0.5) * 0.5
    z0 = np.minimum(np.floor(z).astype(int), n3 - 2)
    f = z - z0
    col = vol.astype(np.float64)
    vals = (1 - f)[:, None, None] * col[z0] + f[:, None, None] * col[z0 + 1]
    m = np.clip((vals - vmin) / (vmax - vmin), 0, 1).max(0)
    return np.repeat(m[..., None], 4, -1)


@pytest.mark.parametrize("window", [(None, None), (-0.5, 2.0)])
def test_axis_columns_match_numpy(orc, window):
    rng = _rng(11)
    n1, n2, n3 = 24, 16, 20
    vol = rng.normal(0, 1, (n3, n2, n1)).astype(np.float32)
    vol[4:8, 2:6, 5:15] += 4.0
    vmin = float(vol.min()) if window[0] is None else window[0]
    vmax = float(vol.max()) if window[1] is None else window[1]
    res = orc.render(vol, synth.tf_ramp(8), [np.eye(3)], n1, n2, vmin, vmax, tau=2.0, extent=float(n1),
                     mode=MIP)
    np.testing.assert_allclose(res["image"][0], _column_mip(vol, vmin, vmax), rtol=0, atol=1e-12)


@pytest.mark.parametrize("seed,boxes", [(21, None), (22, "grid"), (23, "kd")])
def test_exact_rational(orc, seed, boxes):
    rng = _rng(seed)
    dims = (5, 4, 6)
    vol = rng.normal(0, 1, dims[::-1]).astype(np.float32)
    tf = synth.tf_ramp(8)
    R = synth.random_rotation(rng)
    vmin, vmax = -1.0, 1.5
    bl = None
    bricks = None
    if boxes == "grid":
        bl, _ = oracle.grid_boxes(dims, (2, 3, 2))
        bricks = {"grid": (2, 3, 2)}
    elif boxes == "kd":
        bl = oracle.kd_boxes(dims, 3)
        bricks = bl
    W = H = 5
    ex = np.array(exact.to_float(exact.render(vol.tolist(), tf.tolist(), R.tolist(), W, H, 6.0, vmin, vmax,
                                              boxes=bl, mip=True)))
    got = orc.render(vol, tf, [R], W, H, vmin, vmax, tau=2.0, extent=6.0, bricks=bricks, mode=MIP)
    assert (got["flags"] & oracle.FLAG_GEOM).sum() == 0
    np.testing.assert_allclose(got["image"][0], ex, rtol=0, atol=1e-12)


def test_bricks_and_termination_change_nothing(orc):
    rng = _rng(31)
    dims = (30, 26, 34)
    vol = synth.cube(*dims, seed=32, n_sources=4, sigma_range=(1.5, 3.0))
    tf = synth.tf_ramp(16)
    vmin, vmax = float(vol.min()), float(vol.max()) - 2.0  # some rays saturate
    views = synth.random_views(3, 33)
    whole = orc.render(vol, tf, views, 24, 24, vmin, vmax, tau=2.0, mode=MIP)["image"]
    for bricks in ({"grid": (8, 10, 12)}, oracle.kd_boxes(dims, 5)):
        b = orc.render(vol, tf, views, 24, 24, vmin, vmax, tau=2.0, bricks=bricks, mode=MIP)["image"]
        assert np.array_equal(b, whole)
    ert = orc.render(vol, tf, views, 24, 24, vmin, vmax, tau=0.5, mode=MIP)["image"]
    assert np.array_equal(ert, whole)
    assert (whole[..., 0] == 1.0).any() and (whole[..., 0] < 1.0).any()
    del rng


def test_roll_180_flips(orc):
    vol = synth.cube(20, 18, 22, seed=41, n_sources=3, sigma_range=(1.5, 3.0))
    R = synth.random_views(1, 42)[0]
    Rroll = np.array([-R[0], -R[1], R[2]])
    a = orc.render(vol, synth.tf_ramp(8), [R], 16, 16, float(vol.min()), float(vol.max()), tau=2.0, mode=MIP)
    b = orc.render(vol, synth.tf_ramp(8), [Rroll], 16, 16, float(vol.min()), float(vol.max()), tau=2.0, mode=MIP)
    np.testing.assert_allclose(a["image"][0], b["image"][0][::-1, ::-1], rtol=0, atol=1e-12)
