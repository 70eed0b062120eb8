"""Sort-last invariants of the FP64 oracle (paper Sec. 2.3 and Sec. 2.5).

* ERT off: compositing the sub-volume images in depth order equals rendering
  the whole volume (the over operator is associative), up to FP64 rounding.
* Local ERT (each sub-volume stops on its own): every channel is within
  1 - tau of the whole-volume result without ERT, because everything behind an
  opacity >= tau contributes at most 1 - tau.
* The partition of the lattice is exact: per-ray sample counts do not depend
  on the bricking.
"""
import numpy as np
import pytest

import synth


def _setup(seed, dims):
    n1, n2, n3 = dims
    vol = synth.cube(n1, n2, n3, seed=seed, n_sources=6, sigma_range=(1.5, 3.0), band=True)
    return vol, float(vol.min()), float(vol.max())


@pytest.mark.parametrize("bricks", [{"grid": (16, 16, 16)}, {"grid": (7, 9, 11)}, "kd5", "kd8"])
def test_bricked_equals_whole_without_ert(orc, bricks):
    dims = (40, 36, 48)
    vol, vmin, vmax = _setup(21, dims)
    if isinstance(bricks, str):
        bricks = orc.kd_boxes(dims, int(bricks[2:]))
    tf = synth.tf_colour(256)
    tf[:, 3] *= 4
    views = synth.random_views(3, 22)
    whole = orc.render(vol, tf, views, 48, 40, vmin, vmax, tau=2.0)
    br = orc.render(vol, tf, views, 48, 40, vmin, vmax, tau=2.0, bricks=bricks)
    ok = (whole["flags"] == 0) & (br["flags"] == 0)
    assert ok.mean() > 0.999
    d = np.abs(whole["image"] - br["image"])[ok]
    assert d.max() <= 1e-12
    assert whole["nsamples"] == br["nsamples"]


@pytest.mark.parametrize("tau", [0.9, 0.99])
def test_local_ert_within_one_minus_tau(orc, tau):
    dims = (40, 36, 48)
    vol, vmin, vmax = _setup(23, dims)
    tf = synth.tf_ramp(256)
    tf[:, 3] = np.minimum(1.0, tf[:, 3] * 40)
    views = synth.random_views(2, 24)
    whole = orc.render(vol, tf, views, 40, 40, vmin, vmax, tau=2.0)["image"]
    loc = orc.render(vol, tf, views, 40, 40, vmin, vmax, tau=tau, bricks={"grid": (12, 12, 12)})
    d = np.abs(whole - loc["image"])
    assert d.max() <= (1 - tau) + 1e-12
    # and ERT actually changed something
    assert d.max() > 1e-4


def test_global_ert_whole_matches_single_chain(orc):
    """Whole-volume ERT: within 1 - tau of the untruncated result, exactly 1 - T >= tau at stops."""
    dims = (30, 30, 30)
    vol, vmin, vmax = _setup(25, dims)
    tf = synth.tf_ramp(256)
    tf[:, 3] = np.minimum(1.0, tf[:, 3] * 15)
    v = synth.random_views(1, 26)
    full = orc.render(vol, tf, v, 32, 32, vmin, vmax, tau=2.0)["image"]
    ert = orc.render(vol, tf, v, 32, 32, vmin, vmax, tau=0.95)["image"]
    assert np.abs(full - ert).max() <= 0.05 + 1e-12
    stopped = ert[..., 3] >= 0.95
    assert stopped.any()


def test_grid_boxes_partition():
    import oracle
    dims = (512, 512, 1024)
    boxes, counts = oracle.grid_boxes(dims, (256, 256, 512))
    assert counts == (2, 2, 2) and len(boxes) == 8
    assert boxes[0] == ((0, 0, 0), (256, 256, 512), (0, 0, 0))
    assert boxes[7] == ((256, 256, 512), (511, 511, 1023), (1, 1, 1))
    b2, c2 = oracle.grid_boxes((2048, 2048, 1536), (256, 256, 256))
    assert c2 == (8, 8, 6) and len(b2) == 384


def test_kd_boxes_cover_domain():
    import oracle
    dims = (100, 60, 80)
    for p in range(1, 10):
        boxes = oracle.kd_boxes(dims, p)
        assert len(boxes) == p
        vol = sum(np.prod([hi[i] - lo[i] for i in range(3)]) for lo, hi, _ in boxes)
        assert vol == 99 * 59 * 79
    b3 = oracle.kd_boxes(dims, 3)
    # first split is across the longest axis (axis 1) at the 1/3 plane
    assert b3[0] == ((0, 0, 0), (33, 59, 79), (0, 1, 1))
