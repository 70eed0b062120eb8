"""Pins of the oracle's spectral-channel mask (weights along axis 3).

* an all-ones mask changes no bit, an all-zero mask blanks the image
  (emission-absorption and MIP, whole and sub-volumes);
* rays down voxel columns (identity view): numpy's linear interpolation of the
  mask and of the table, accumulated with ``np.cumprod``;
* the exact-rational brute force with random masks, whole and in sub-volumes,
  emission-absorption and MIP.
"""
import numpy as np
import pytest

import oracle
import synth
from oracle import exact


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def test_ones_and_zeros(orc):
    dims = (30, 26, 34)
    vol = synth.cube(*dims, seed=141, n_sources=4, sigma_range=(1.5, 3.0))
    tf = synth.tf_colour(64)
    views = synth.random_views(3, 142)
    mn, mx = float(vol.min()), float(vol.max())
    for mode in (oracle.MODE_DVR, oracle.MODE_MIP):
        for bricks in (None, {"grid": (8, 10, 12)}):
            base = orc.render(vol, tf, views, 24, 20, mn, mx, tau=0.9, bricks=bricks, mode=mode)["image"]
            ones = orc.render(vol, tf, views, 24, 20, mn, mx, tau=0.9, bricks=bricks, mode=mode,
                              mask=np.ones(dims[2], np.float32))["image"]
            zeros = orc.render(vol, tf, views, 24, 20, mn, mx, tau=0.9, bricks=bricks, mode=mode,
                               mask=np.zeros(dims[2], np.float32))["image"]
            assert np.array_equal(base, ones)
            assert (zeros == 0).all() and (base > 0).any()


def _column_render(vol, tf, vmin, vmax, mask):
    """Identity view, one ray per voxel column, no termination: samples at
    z = (k + 1/2)/2, value and mask by ``np.interp`` along the column, table by
    ``np.interp``, accumulation by ``np.cumprod``."""
    n3, n2, n1 = vol.shape
    M = tf.shape[0]
    z = (np.arange(2 * (n3 - 1)) + 0.5) * 0.5
    col = vol.astype(np.float64).reshape(n3, -1)
    vals = np.stack([np.interp(z, np.arange(n3), col[:, i]) for i in range(col.shape[1])], -1)
    m = np.interp(z, np.arange(n3), mask.astype(np.float64))[:, None]
    u = np.clip((vals - vmin) / (vmax - vmin), 0, 1) * (M - 1)
    rgba = np.stack([np.interp(u, np.arange(M), tf[:, c].astype(np.float64)) for c in range(4)], -1)
    a = rgba[..., 3] * m
    T = np.cumprod(1 - a, axis=0)
    Tprev = np.concatenate([np.ones((1, a.shape[1])), T[:-1]], axis=0)
    C = (Tprev[..., None] * a[..., None] * rgba[..., :3]).sum(0)
    return np.concatenate([C, (1 - T[-1])[..., None]], -1).reshape(n2, n1, 4)


@pytest.mark.parametrize("kind", ["band", "random"])
def test_axis_columns_match_numpy(orc, kind):
    rng = _rng(143)
    n1, n2, n3 = 20, 12, 26
    vol = rng.normal(0, 1, (n3, n2, n1)).astype(np.float32)
    vol[6:12, 3:7, 5:15] += 5.0
    tf = synth.tf_colour(64)
    tf[:, 3] *= 4.0
    if kind == "band":
        mask = np.ones(n3, np.float32)
        mask[8:15] = 0.0  # channels switched off
    else:
        mask = rng.uniform(0, 1, n3).astype(np.float32)
    vmin, vmax = float(vol.min()), float(vol.max())
    res = orc.render(vol, tf, [np.eye(3)], n1, n2, vmin, vmax, tau=2.0, extent=float(n1), mask=mask)
    np.testing.assert_allclose(res["image"][0], _column_render(vol, tf, vmin, vmax, mask), rtol=0, atol=1e-12)


@pytest.mark.parametrize("seed,boxes,mip", [(151, None, False), (152, "grid", False), (153, "kd", True),
                                            (154, None, True)])
def test_exact_rational(orc, seed, boxes, mip):
    rng = _rng(seed)
    dims = (5, 4, 6)
    vol = rng.normal(0, 1, dims[::-1]).astype(np.float32)
    tf = rng.uniform(0, 1, (8, 4)).astype(np.float32)
    tf[:, 3] *= 0.4
    mask = rng.uniform(0, 1, dims[2]).astype(np.float32)
    mask[2] = 0.0
    R = synth.random_rotation(rng)
    bl = bricks = None
    if boxes == "grid":
        bl, _ = oracle.grid_boxes(dims, (2, 3, 2))
        bricks = {"grid": (2, 3, 2)}
    elif boxes == "kd":
        bl = bricks = oracle.kd_boxes(dims, 3)
    vmin, vmax = float(vol.min()) + 0.2, float(vol.max()) - 0.2
    ex = np.array(exact.to_float(exact.render(vol.tolist(), tf.tolist(), R.tolist(), 5, 5, 6.0, vmin, vmax,
                                              tau=0.8, boxes=bl, mip=mip, mask=mask.tolist())))
    got = orc.render(vol, tf, [R], 5, 5, vmin, vmax, tau=0.8, extent=6.0, bricks=bricks,
                     mode=oracle.MODE_MIP if mip else oracle.MODE_DVR, mask=mask)
    assert (got["flags"] & oracle.FLAG_GEOM).sum() == 0
    np.testing.assert_allclose(got["image"][0], ex, rtol=0, atol=1e-12)
