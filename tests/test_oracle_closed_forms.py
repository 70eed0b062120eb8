"""Pins of the FP64 oracle against closed forms, library routines and invariants.

None of these re-types the oracle's own loops: each expected value comes from
a closed form (constant cube), an independent formulation built from numpy
primitives (axis-aligned rays through voxel columns: ``np.interp`` +
``np.cumprod``), a symmetry of the orthographic camera, or exact algebra of
the over operator (paper Sec. 2.5: the blending operator is associative).
"""
import math

import numpy as np
import pytest

import synth

pytestmark = []


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


# ----------------------------------------------------------------- constant cube
def _const_tf(a, rgb=(0.25, 0.5, 0.75)):
    # three entries; s = 1/2 lands exactly on the middle entry
    return np.array([[0, 0, 0, 0], [rgb[0], rgb[1], rgb[2], a], [1, 1, 1, 0.5]], np.float32)


@pytest.mark.parametrize("n", [16, 33])
def test_constant_cube_axis_rays(orc, n):
    """Axis rays through an n^3 constant cube: n_k = 2(n-1) samples, A = 1-(1-a)^n_k, C = rgb A."""
    a = 0.03125
    tf = _const_tf(a)
    vol = np.full((n, n, n), 0.5, np.float32)
    W = H = 8
    res = orc.render(vol, tf, [np.eye(3)], W, H, vmin=0.0, vmax=1.0, tau=2.0, extent=float(n - 1))
    img = res["image"][0]
    k = 2 * (n - 1)
    A = 1.0 - (1.0 - a) ** k
    np.testing.assert_allclose(img[..., 3], A, rtol=0, atol=1e-13)
    for c, rgb in enumerate((0.25, 0.5, 0.75)):
        np.testing.assert_allclose(img[..., c], rgb * A, rtol=0, atol=1e-13)
    assert res["nsamples"] == W * H * k


@pytest.mark.parametrize("tau", [0.5, 0.9, 0.99])
def test_constant_cube_ert(orc, tau):
    """With ERT the ray stops after n_eff = min(n, ceil(log(1-tau)/log(1-a))) samples."""
    n = 40
    a = 0.0625
    vol = np.full((n, n, n), 0.5, np.float32)
    res = orc.render(vol, _const_tf(a), [np.eye(3)], 4, 4, 0.0, 1.0, tau=tau, extent=float(n - 1))
    k = 2 * (n - 1)
    neff = min(k, math.ceil(math.log(1 - tau) / math.log(1 - a)))
    A = 1.0 - (1.0 - a) ** neff
    np.testing.assert_allclose(res["image"][0][..., 3], A, atol=1e-13)


def test_constant_cube_any_view_counts(orc):
    """Any view: each pixel is 1-(1-a)^k for its own integer k, and sum k ~ V/(p^2 step)."""
    n1, n2, n3 = 30, 24, 40
    a = 0.0078125
    vol = np.full((n3, n2, n1), 0.5, np.float32)
    W, H = 96, 80
    R = synth.random_views(1, 77)[0]
    res = orc.render(vol, _const_tf(a), [R], W, H, 0.0, 1.0, tau=2.0)
    A = res["image"][0][..., 3]
    k = np.log1p(-A) / math.log1p(-a)
    assert np.allclose(k, np.round(k), atol=1e-6)
    S = math.sqrt((n1 - 1) ** 2 + (n2 - 1) ** 2 + (n3 - 1) ** 2)
    pitch = S / W
    vbox = (n1 - 1) * (n2 - 1) * (n3 - 1)
    expect = vbox / (pitch * pitch * 0.5)
    hit = int((A > 0).sum())
    # per ray the count is within 1/2 of chord/step; pixel-area discretisation adds
    # at most the boundary strip (perimeter of the projected box, about 2 px wide)
    assert abs(res["nsamples"] - expect) <= 0.5 * hit + 0.03 * expect
    assert res["nsamples"] == int(np.round(k).sum())


# -------------------------------------------------- axis columns via numpy
def _column_render(vol, tf, vmin, vmax, tau):
    """Image for R = I, W = n1, H = n2, extent = n1: each ray runs down one voxel column.

    Samples sit at z = (k + 1/2)/2; values are linear interpolation along z;
    the table lookup is ``np.interp`` and the accumulation ``np.cumprod``.
    """
    n3, n2, n1 = vol.shape
    M = tf.shape[0]
    nk = 2 * (n3 - 1)
    z = (np.arange(nk) + 0.5) * 0.5
    z0 = np.minimum(np.floor(z).astype(int), n3 - 2)
    f = z - z0
    col = vol.astype(np.float64)
    vals = (1 - f)[:, None, None] * col[z0] + f[:, None, None] * col[z0 + 1]  # [nk][n2][n1]
    s = np.clip((vals - vmin) / (vmax - vmin), 0, 1)
    u = s * (M - 1)
    rgba = np.stack([np.interp(u, np.arange(M), tf[:, c].astype(np.float64)) for c in range(4)], -1)
    a = rgba[..., 3]
    T = np.cumprod(1 - a, axis=0)
    Tprev = np.concatenate([np.ones((1, n2, n1)), T[:-1]], axis=0)
    contrib = Tprev[..., None] * a[..., None] * rgba[..., :3]
    if tau < 1:
        stop = (1 - T) >= tau
        first = np.where(stop.any(0), stop.argmax(0), nk - 1)
        keep = np.arange(nk)[:, None, None] <= first[None]
        C = (contrib * keep[..., None]).sum(0)
        Tend = np.take_along_axis(T, first[None], 0)[0]
    else:
        C = contrib.sum(0)
        Tend = T[-1]
    return np.concatenate([C, (1 - Tend)[..., None]], -1)


@pytest.mark.parametrize("tau", [2.0, 0.6])
def test_axis_columns_match_numpy(orc, tau):
    rng = _rng(5)
    n1, n2, n3 = 32, 16, 24
    vol = rng.normal(0, 1, (n3, n2, n1)).astype(np.float32)
    vol[5:9, 3:7, 10:20] += 6.0
    tf = synth.tf_colour(64)
    tf[:, 3] *= 5.0  # make opacity large enough to terminate
    vmin, vmax = float(vol.min()), float(vol.max())
    res = orc.render(vol, tf, [np.eye(3)], n1, n2, vmin, vmax, tau=tau, extent=float(n1),
                     ert_margin=0.0)
    want = _column_render(vol, tf, vmin, vmax, tau)
    np.testing.assert_allclose(res["image"][0], want, rtol=0, atol=1e-12)


def test_view_along_axis1_is_transposed_columns(orc):
    """Rows of R are the view axes: R = cyclic permutation looks down axis 1."""
    rng = _rng(6)
    n1, n2, n3 = 12, 16, 8
    vol = rng.normal(0, 1, (n3, n2, n1)).astype(np.float32)
    tf = synth.tf_colour(32)
    vmin, vmax = float(vol.min()), float(vol.max())
    R = np.array([[0, 1, 0], [0, 0, 1], [1, 0, 0]], np.float64)  # image x = axis 2, y = axis 3
    res = orc.render(vol, tf, [R], n2, n3, vmin, vmax, tau=2.0, extent=float(n2))
    volT = np.ascontiguousarray(vol.transpose(2, 0, 1))  # new axes (1,2,3) = old (2,3,1)
    want = _column_render(volT, tf, vmin, vmax, 2.0)
    np.testing.assert_allclose(res["image"][0], want, rtol=0, atol=1e-12)


# --------------------------------------------------------- camera symmetries
def test_roll_180_flips_image(orc):
    rng = _rng(7)
    vol = rng.normal(0, 1, (20, 18, 22)).astype(np.float32)
    tf = synth.tf_colour(64)
    R = synth.random_views(1, 8)[0]
    R2 = np.diag([-1.0, -1.0, 1.0]) @ R
    W, H = 40, 30
    a = orc.render(vol, tf, [R], W, H, float(vol.min()), float(vol.max()), tau=0.95)
    b = orc.render(vol, tf, [R2], W, H, float(vol.min()), float(vol.max()), tau=0.95)
    ok = (a["flags"][0] == 0) & (b["flags"][0][::-1, ::-1] == 0)
    diff = np.abs(a["image"][0] - b["image"][0][::-1, ::-1])
    assert diff[ok].max() <= 1e-12
    assert ok.mean() > 0.9


def test_roll_90_rotates_image(orc):
    rng = _rng(9)
    vol = rng.normal(0, 1, (14, 18, 16)).astype(np.float32)
    tf = synth.tf_colour(64)
    R = synth.random_views(1, 10)[0]
    Rr = np.array([[0, 1, 0], [-1, 0, 0], [0, 0, 1]], np.float64) @ R
    W = H = 36
    a = orc.render(vol, tf, [R], W, H, float(vol.min()), float(vol.max()), tau=2.0)["image"][0]
    b = orc.render(vol, tf, [Rr], W, H, float(vol.min()), float(vol.max()), tau=2.0)["image"][0]
    # pixel (u', v') of the rolled view shows pixel (W-1-v', u') of the original
    want = np.empty_like(a)
    for v2 in range(H):
        for u2 in range(W):
            want[v2, u2] = a[u2, W - 1 - v2]
    np.testing.assert_allclose(b, want, atol=1e-12)


def test_window_degenerate_gives_entry0(orc):
    """vmax == vmin gives s = 0: every sample takes table entry 0."""
    vol = _rng(3).normal(0, 1, (10, 10, 10)).astype(np.float32)
    tf = np.array([[0.5, 0.25, 1.0, 0.125], [1, 1, 1, 1]], np.float32)
    res = orc.render(vol, tf, [np.eye(3)], 8, 8, 1.0, 1.0, tau=2.0, extent=9.0)
    img = res["image"][0]
    k = 2 * 9
    A = 1 - (1 - 0.125) ** k
    inside = img[..., 3] > 0
    np.testing.assert_allclose(img[inside][:, 3], A, atol=1e-13)
    np.testing.assert_allclose(img[inside][:, 0], 0.5 * A, atol=1e-13)


def test_miss_outside_and_background_zero(orc):
    vol = np.ones((8, 8, 8), np.float32)
    tf = synth.tf_ramp(16)
    res = orc.render(vol, tf, [np.eye(3)], 16, 16, 0.0, 2.0, tau=2.0, extent=40.0)
    img = res["image"][0]
    # pixel pitch 2.5 voxels: the 7-voxel box covers the central pixels only
    assert (img[0] == 0).all() and (img[:, 0] == 0).all()
    assert (img[8, 8, 3] > 0)


# ----------------------------------------------------------- compositing algebra
def _rand_layers(rng, n, shape):
    """n random premultiplied RGBA layers (colour <= opacity)."""
    out = []
    for _ in range(n):
        a = rng.uniform(0, 1, shape + (1,))
        out.append(np.concatenate([rng.uniform(0, 1, shape + (3,)) * a, a], -1))
    return np.stack(out)


def test_over_associative(orc):
    rng = _rng(11)
    X, Y, Z = _rand_layers(rng, 3, (50,))
    xy = orc.composite(np.stack([X, Y]))
    yz = orc.composite(np.stack([Y, Z]))
    left = orc.composite(np.stack([xy, Z]))
    right = orc.composite(np.stack([X, yz]))
    allthree = orc.composite(np.stack([X, Y, Z]))
    np.testing.assert_allclose(left, right, atol=1e-15)
    np.testing.assert_allclose(left, allthree, atol=1e-15)


def test_over_identity_and_opaque_front(orc):
    rng = _rng(12)
    X, Y = _rand_layers(rng, 2, (40,))
    zero = np.zeros_like(X)
    np.testing.assert_array_equal(orc.composite(np.stack([X, zero])), X)
    np.testing.assert_array_equal(orc.composite(np.stack([zero, X])), X)
    F = X.copy()
    F[:, 3] = 1.0
    np.testing.assert_array_equal(orc.composite(np.stack([F, Y])), F)


def test_over_two_constant_layers(orc):
    """Two layers of opacity A1, A2: A = 1 - (1-A1)(1-A2), C = C1 + (1-A1) C2."""
    L1 = np.array([[0.1, 0.2, 0.3, 0.4]])
    L2 = np.array([[0.5, 0.25, 0.125, 0.75]])
    out = orc.composite(np.stack([L1, L2]))[0]
    assert out[3] == pytest.approx(1 - 0.6 * 0.25, abs=1e-15)
    np.testing.assert_allclose(out[:3], L1[0, :3] + 0.6 * L2[0, :3], atol=1e-15)


# ----------------------------------------------------------------- min / max
def test_minmax_matches_numpy(orc):
    x = _rng(13).normal(0, 3, 100003).astype(np.float32)
    mn, mx, bad = orc.minmax(x)
    assert mn == float(x.min()) and mx == float(x.max()) and bad == 0
    x[17] = np.nan
    x[99] = np.inf
    mn2, mx2, bad2 = orc.minmax(x)
    assert bad2 == 2


def test_box_minmax_matches_numpy(orc):
    v = _rng(14).normal(0, 1, (9, 10, 11)).astype(np.float32)
    mn, mx = orc.box_minmax(v, (2, 3, 1), (7, 8, 5))
    sub = v[1:6, 3:9, 2:8]
    assert mn == float(sub.min()) and mx == float(sub.max())


@pytest.mark.parametrize("tau", [0.5, 0.99, 2.0])
def test_constant_cube_evaluated_samples(orc, tau):
    """Evaluated samples per ray: n_eff = min(n, ceil(log(1-tau)/log(1-a))) on axis rays
    (all n without early termination); with two sub-volumes along the ray each stops on
    its own, so the count is the sum of the two chains' closed forms."""
    n = 40
    a = 0.0625
    vol = np.full((n, n, n), 0.5, np.float32)
    k = 2 * (n - 1)
    ys, xs = np.meshgrid(np.arange(1, 4), np.arange(1, 4), indexing="ij")
    rv = np.zeros(ys.size, np.int32)
    res = orc.render_rays(vol, _const_tf(a), [np.eye(3)], 4, 4, rv, xs.ravel(), ys.ravel(), 0.0, 1.0, tau=tau,
                          extent=float(n - 1))
    stop = k if tau >= 1 else min(k, math.ceil(math.log(1 - tau) / math.log(1 - a)))
    assert (res["nsamples"] == k).all()
    assert (res["neval"] == stop).all()
    # two sub-volumes split at z = 20: 40 samples in the front one, 38 behind
    boxes = [((0, 0, 0), (n - 1, n - 1, 20), (1, 1, 0)), ((0, 0, 20), (n - 1, n - 1, n - 1), (1, 1, 1))]
    res = orc.render_rays(vol, _const_tf(a), [np.eye(3)], 4, 4, rv, xs.ravel(), ys.ravel(), 0.0, 1.0, tau=tau,
                          extent=float(n - 1), bricks=boxes)
    per = [40, k - 40]
    want = sum(c if tau >= 1 else min(c, math.ceil(math.log(1 - tau) / math.log(1 - a))) for c in per)
    assert (res["neval"] == want).all()
