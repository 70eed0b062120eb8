"""FP64 oracle vs the exact-rational brute force on tiny inputs.

The brute force (``oracle/exact.py``) evaluates the same definition with
``fractions.Fraction`` and no rounding, sample by sample, with a per-ray sort
of the sub-volume results; forward-mode dual numbers give exact directional
derivatives.  Agreement to 1e-12 pins the FP64 oracle's camera, ray/box,
lattice, trilinear, table, accumulation, ERT, ownership and ordering steps;
the dual-number check pins its reverse-mode gradient.
"""
import numpy as np
import pytest

import synth
from oracle import exact


def _case(seed, dims=(5, 4, 6), M=8, amax=0.3):
    rng = np.random.Generator(np.random.PCG64(seed))
    n1, n2, n3 = dims
    vol = rng.normal(0, 1, (n3, n2, n1)).astype(np.float32)
    tf = rng.uniform(0, 1, (M, 4)).astype(np.float32)
    tf[:, 3] *= amax
    R = synth.random_rotation(rng)
    return vol, tf, R


def _exact_image(vol, tf, R, W, H, extent, vmin, vmax, tau, boxes=None):
    img = exact.render(vol.tolist(), tf.tolist(), R.tolist(), W, H, extent, vmin, vmax,
                       step=0.5, tau=tau, boxes=boxes)
    return np.array(exact.to_float(img))


@pytest.mark.parametrize("seed,tau", [(1, 2.0), (2, 0.7), (3, 0.5), (4, 0.9)])
def test_whole_volume_matches_exact(orc, seed, tau):
    vol, tf, R = _case(seed)
    vmin, vmax = float(vol.min()) + 0.25, float(vol.max()) - 0.25  # exercise both clamps
    W, H, ext = 6, 5, 6.0
    res = orc.render(vol, tf, [R], W, H, vmin, vmax, tau=tau, extent=ext)
    want = _exact_image(vol, tf, R, W, H, ext, vmin, vmax, tau)
    ok = (res["flags"][0] & orc.FLAG_GEOM) == 0
    assert ok.all()
    np.testing.assert_allclose(res["image"][0], want, rtol=0, atol=1e-12)
    assert (want[..., 3] > 0).sum() >= 12


@pytest.mark.parametrize("seed,tau,kind", [(5, 2.0, "grid"), (6, 0.6, "grid"), (7, 0.8, "kd"),
                                           (8, 2.0, "kd")])
def test_bricked_matches_exact(orc, seed, tau, kind):
    dims = (6, 5, 7)
    vol, tf, R = _case(seed, dims=dims)
    vmin, vmax = float(vol.min()), float(vol.max())
    W, H, ext = 6, 6, 9.0
    if kind == "grid":
        bs = (2, 3, 4)
        boxes, _ = orc.grid_boxes(dims, bs)
        bricks = {"grid": bs}
    else:
        boxes = orc.kd_boxes(dims, 3)
        bricks = boxes
    res = orc.render(vol, tf, [R], W, H, vmin, vmax, tau=tau, extent=ext, bricks=bricks)
    want = _exact_image(vol, tf, R, W, H, ext, vmin, vmax, tau, boxes=boxes)
    ok = (res["flags"][0] & orc.FLAG_GEOM) == 0
    assert ok.all()
    np.testing.assert_allclose(res["image"][0], want, rtol=0, atol=1e-12)


def test_axis_aligned_rational_view(orc):
    """A view with exactly representable pixel centres (axis-aligned, extent a power of two)."""
    vol, tf, _ = _case(9, dims=(4, 5, 6))
    R = np.array([[0, 0, 1], [1, 0, 0], [0, 1, 0]], np.float64)
    vmin, vmax = float(vol.min()), float(vol.max())
    res = orc.render(vol, tf, [R], 8, 8, vmin, vmax, tau=0.8, extent=8.0)
    want = _exact_image(vol, tf, R, 8, 8, 8.0, vmin, vmax, 0.8)
    np.testing.assert_allclose(res["image"][0], want, rtol=0, atol=1e-12)


@pytest.mark.parametrize("seed,tau", [(10, 2.0), (11, 0.75)])
def test_gradient_matches_exact_directional_derivative(orc, seed, tau):
    """<grad, dir> from the FP64 reverse-mode gradient == exact forward-mode derivative."""
    vol, tf, R = _case(seed, dims=(4, 5, 5), M=6)
    rng = np.random.Generator(np.random.PCG64(seed + 100))
    vmin, vmax = float(vol.min()) + 0.1, float(vol.max()) - 0.1
    W, H, ext = 5, 4, 7.0
    g = rng.normal(0, 1, (H, W, 4))
    dvol = rng.normal(0, 1, vol.shape)
    dtf = rng.normal(0, 1, tf.shape)
    gtf, gvol, img = orc.render_grad(vol, tf, R, W, H, g, vmin, vmax, tau=tau, extent=ext)
    dual = exact.render(vol.tolist(), tf.tolist(), R.tolist(), W, H, ext, vmin, vmax, tau=tau,
                        dvol=dvol.tolist(), dtf=dtf.tolist())
    arr = np.array(exact.to_float(dual))  # [H][W][4][2] (value, derivative)
    np.testing.assert_allclose(img, arr[..., 0], atol=1e-12)
    want = float((g * arr[..., 1]).sum())
    got = float((gtf * dtf).sum() + (gvol * dvol).sum())
    assert got == pytest.approx(want, rel=1e-10, abs=1e-12)
