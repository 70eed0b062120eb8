"""Pins of the FP64 oracle's exact gradient (the adjoint's reference).

* central finite differences of the FP64 forward (eps = 1e-4) for every
  transfer-function entry and for sampled voxels;
* the dot-product (adjoint) identity against a finite-difference directional
  derivative over all voxels and table entries at once;
* a constant cube where dA/da = n (1 - a)^(n-1) and only the two table
  entries around s receive gradient.
"""
import math

import numpy as np
import pytest

import synth


def _loss(orc, vol, tf, views, W, H, vmin, vmax, target):
    r = orc.render(vol, tf, views, W, H, vmin, vmax, tau=2.0)
    return 0.5 * float(((r["image"] - target) ** 2).sum())


def _case():
    dims = (12, 10, 14)
    vol = synth.cube(*dims, seed=31, n_sources=3, sigma_range=(1.5, 2.5), band=True)
    vmin, vmax = float(vol.min()) - 1.0, float(vol.max()) + 1.0  # no clamping: smooth in voxels
    tf = synth.tf_colour(16)
    tf[:, 3] *= 6
    views = synth.random_views(2, 32)
    W = H = 10
    target_tf = synth.tf_perturbed(tf, 33)
    target = np.stack([
        __import__("oracle").render(vol, target_tf, [v], W, H, vmin, vmax, tau=2.0)["image"][0]
        for v in views])
    return vol, tf, views, W, H, vmin, vmax, target


def _grad(orc, vol, tf, views, W, H, vmin, vmax, target):
    gtf = np.zeros(tf.shape)
    gvol = np.zeros(vol.shape)
    for j, v in enumerate(views):
        img = orc.render(vol, tf, [v], W, H, vmin, vmax, tau=2.0)["image"][0]
        a, b, _ = orc.render_grad(vol, tf, v, W, H, img - target[j], vmin, vmax)
        gtf += a
        gvol += b
    return gtf, gvol


def _rel(g, fd):
    scale = max(1e-3 * np.abs(fd).max(), 1e-12)
    return np.abs(g - fd) / np.maximum(np.abs(fd), scale)


def test_tf_gradient_vs_central_fd(orc):
    vol, tf, views, W, H, vmin, vmax, target = _case()
    gtf, _ = _grad(orc, vol, tf, views, W, H, vmin, vmax, target)
    # FP64 forward: eps = 1e-4 keeps the O(eps^2) truncation of central differences
    # (about 2e-3 relative at eps = 1e-3 for the opacity entries here) well below 1e-3
    eps = 1e-4
    fd = np.zeros_like(gtf)
    tf64 = tf.astype(np.float64)
    for i in range(tf.shape[0]):
        for c in range(4):
            tp, tm = tf64.copy(), tf64.copy()
            tp[i, c] += eps
            tm[i, c] -= eps
            # the oracle reads float32 tables: perturb in a way float32 represents exactly
            tp32, tm32 = tp.astype(np.float32), tm.astype(np.float32)
            h = float(tp32[i, c]) - float(tm32[i, c])
            fd[i, c] = (_loss(orc, vol, tp32, views, W, H, vmin, vmax, target)
                        - _loss(orc, vol, tm32, views, W, H, vmin, vmax, target)) / h
    assert _rel(gtf, fd).max() <= 1e-3


def test_voxel_gradient_vs_central_fd(orc):
    vol, tf, views, W, H, vmin, vmax, target = _case()
    _, gvol = _grad(orc, vol, tf, views, W, H, vmin, vmax, target)
    rng = np.random.Generator(np.random.PCG64(34))
    nz = np.argwhere(np.abs(gvol) > 1e-6 * np.abs(gvol).max())
    pick = nz[rng.choice(len(nz), size=min(40, len(nz)), replace=False)]
    eps = 1e-3
    for z, y, x in pick:
        vp, vm = vol.copy(), vol.copy()
        vp[z, y, x] += eps
        vm[z, y, x] -= eps
        h = float(vp[z, y, x]) - float(vm[z, y, x])
        fd = (_loss(orc, vp, tf, views, W, H, vmin, vmax, target)
              - _loss(orc, vm, tf, views, W, H, vmin, vmax, target)) / h
        g = gvol[z, y, x]
        assert abs(g - fd) <= 1e-3 * max(abs(fd), 1e-3 * np.abs(gvol).max()), (z, y, x, g, fd)


def test_dot_product_identity(orc):
    """<J^T w, d> from the adjoint == directional derivative (FD, FP64) along d."""
    vol, tf, views, W, H, vmin, vmax, _ = _case()
    rng = np.random.Generator(np.random.PCG64(35))
    w = rng.normal(0, 1, (len(views), H, W, 4))
    dvol = rng.normal(0, 1, vol.shape)
    gtf = np.zeros(tf.shape)
    gvol = np.zeros(vol.shape)
    for j, v in enumerate(views):
        a, b, _ = orc.render_grad(vol, tf, v, W, H, w[j], vmin, vmax)
        gtf += a
        gvol += b
    eps = 1e-2

    def f(s):
        # volume perturbed in float64 then stored as float32 would add rounding noise;
        # use a scaled copy so the perturbation is exact enough at this eps
        v2 = (vol.astype(np.float64) + s * dvol).astype(np.float32)
        r = orc.render(v2, tf, views, W, H, vmin, vmax, tau=2.0)["image"]
        return float((w * r).sum())

    fd = (f(eps) - f(-eps)) / (2 * eps)
    got = float((gvol * dvol).sum())
    assert got == pytest.approx(fd, rel=2e-3)


def test_constant_cube_gradient_closed_form(orc):
    """Constant cube, axis rays, loss = sum(A): dL/dalpha_table hits exactly the sampled entry."""
    n = 12
    a = 0.0625
    tf = np.array([[0, 0, 0, 0], [0.25, 0.5, 0.75, a], [1, 1, 1, 0.5]], np.float32)
    vol = np.full((n, n, n), 0.5, np.float32)
    W = H = 4
    g = np.zeros((H, W, 4))
    g[..., 3] = 1.0
    gtf, _, img = orc.render_grad(vol, tf, np.eye(3), W, H, g, 0.0, 1.0, extent=float(n - 1))
    k = 2 * (n - 1)
    dA = k * (1 - a) ** (k - 1)
    # s = 1/2 -> u = 1 exactly -> i = 1, w = 0: all gradient on entry 1
    assert gtf[1, 3] == pytest.approx(W * H * dA, rel=1e-12)
    assert np.abs(gtf[0]).max() == 0 and np.abs(gtf[2]).max() == 0
    np.testing.assert_allclose(gtf[1, :3], 0, atol=0)
