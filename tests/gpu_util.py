"""Helpers shared by the GPU tests: device context, parity assertion."""
import numpy as np

import oracle

TOL = 2e-5  # max-abs pixel error, FP32 renderer vs FP64 oracle


def parity(gpu, ref, tol=TOL, max_geom_frac=1e-3, label=""):
    """Compare GPU pixels with oracle pixels.

    gpu: float array [..., 4]; ref: dict from oracle.render / render_rays.
    Pixels whose oracle result lies in an early-termination tie window are
    allowed the extra tolerance the oracle reports (the candidate results of
    stopping one sample earlier or later); pixels decided within rounding of a
    face (flag GEOM) are counted and bounded loosely.
    Returns a summary dict.
    """
    g = np.asarray(gpu, np.float64)
    r = ref["image"]
    extra = ref["tol"]
    flags = ref["flags"]
    geom = (flags & oracle.FLAG_GEOM) != 0
    ert = (flags & oracle.FLAG_ERT) != 0
    diff = np.abs(g - r)
    excess = diff - extra
    strict = ~geom
    worst = float(excess[strict].max()) if strict.any() else 0.0
    worst_plain = float(diff[strict & ~ert].max()) if (strict & ~ert).any() else 0.0
    if worst > tol:
        idx = np.unravel_index(np.argmax(np.where(strict[..., None], excess, -1)), excess.shape)
        raise AssertionError(f"{label}: max |gpu - oracle| beyond tie windows = {worst:.3g} > {tol} at {idx}: "
                             f"gpu {g[idx[:-1]]} oracle {r[idx[:-1]]} extra {extra[idx[:-1]]}")
    nge = int(geom.sum())
    assert nge <= max(2, max_geom_frac * geom.size), f"{label}: {nge} geometric near-tie pixels"
    if nge:
        assert float(diff[geom].max()) <= 0.05, f"{label}: geometric tie pixel off by {diff[geom].max():.3g}"
    return dict(worst=worst, worst_plain=worst_plain, n_ert=int(ert.sum()), n_geom=nge, n=int(flags.size))
