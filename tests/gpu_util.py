"""Helpers shared by the GPU tests: device context, parity assertion."""
import numpy as np

import oracle

TOL = 2e-5  # max-abs pixel error, FP32 renderer vs FP64 oracle


def parity(gpu, ref, tol=TOL, max_geom_frac=1e-3, label=""):
    """Compare GPU pixels with oracle pixels.

    gpu: float array [..., 4]; ref: dict from oracle.render / render_rays.
    Every pixel must match an oracle image within ``tol`` in every channel:
    the oracle's own, or -- for a pixel whose early termination is a tie
    (opacity within rounding of tau, flag ERT) -- one of the valid images the
    oracle lists for it (one per combination of valid stopping samples), all
    four channels from the same image.  Pixels decided within rounding of a
    face (flag GEOM) are counted and bounded loosely.
    Returns a summary dict.
    """
    g = np.asarray(gpu, np.float64)
    flags = ref["flags"]
    geom = (flags & oracle.FLAG_GEOM) != 0
    ert = (flags & oracle.FLAG_ERT) != 0
    err = oracle.match_error(g, ref)
    strict = ~geom
    over = int((ref["ties"]["ncand"] < 0).sum())
    assert over == 0, f"{label}: {over} pixels with more valid images than the oracle lists"
    worst = float(err[strict].max()) if strict.any() else 0.0
    worst_plain = float(err[strict & ~ert].max()) if (strict & ~ert).any() else 0.0
    if worst > tol:
        idx = np.unravel_index(np.argmax(np.where(strict, err, -1)), err.shape)
        raise AssertionError(f"{label}: max |gpu - oracle| = {worst:.3g} > {tol} at {idx} "
                             f"(tie: {bool(ert[idx])}): gpu {g[idx]} oracle {ref['image'][idx]}")
    nge = int(geom.sum())
    assert nge <= max(2, max_geom_frac * geom.size), f"{label}: {nge} geometric near-tie pixels"
    if nge:
        dg = np.abs(g - ref["image"])[geom]
        assert float(dg.max()) <= 0.05, f"{label}: geometric tie pixel off by {dg.max():.3g}"
    return dict(worst=worst, worst_plain=worst_plain, n_ert=int(ert.sum()), n_geom=nge, n=int(flags.size))
