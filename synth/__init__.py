"""Seeded synthetic inputs: spectral cubes, views and transfer-function tables.

These generators produce the inputs of the renderer and nothing else. They hold
none of the rendering arithmetic (no rays, no sampling, no compositing), so the
FP64 oracle and the HIP path can both be fed from here without sharing code.

Cube recipe (a stand-in for the radio survey cubes of the paper's dataset
table: noise-dominated data with compact sources that are elongated along the
spectral axis and a smooth Galactic-plane-like emission band):

* noise: i.i.d. N(0, 1), drawn in float32, one PCG64 stream per z-slab so the
  bits do not depend on the number of worker threads;
* sources: amplitude ~U[5, 20], centre ~U over the cube, sigma_1 = sigma_2 ~U
  over ``sigma_range``, sigma_3 = 3 sigma_1, evaluated in float64 within
  +-4 sigma and added in source order;
* band (optional): amplitude 3, Gaussian across axis 2 with sigma n2/64 centred
  on n2/2 + (n2/8) sin(2 pi x / n1), ripple 1 + 0.2 cos(2 pi z / (n3/4)).

Arrays are C-ordered ``[n3][n2][n1]`` float32 (axis 1 fastest, axis 3
spectral), matching FITS axis order.
"""
from __future__ import annotations

import math
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

__all__ = [
    "cube", "CONFIGS", "config_cube", "config_sources", "rot_axis", "c1_views", "random_views",
    "random_rotation", "tf_ramp", "tf_colour", "tf_noise_suppress", "tf_random",
    "tf_perturbed", "batch_requests", "threads",
]


def threads() -> int:
    """Worker threads for generation: the process's CPU share, capped at 16."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def _source_params(rng, count, shape, sigma_range, margin):
    n3, n2, n1 = shape
    out = []
    for _ in range(count):
        amp = rng.uniform(5.0, 20.0)
        if margin is None:
            c = (rng.uniform(0, n1 - 1), rng.uniform(0, n2 - 1), rng.uniform(0, n3 - 1))
        else:
            c = (rng.uniform(margin, n1 - 1 - margin), rng.uniform(margin, n2 - 1 - margin),
                 rng.uniform(margin, n3 - 1 - margin))
        s1 = rng.uniform(*sigma_range)
        out.append((amp, c, (s1, s1, 3.0 * s1)))
    return out


def _add_source_to_slab(slab, z0, z1, shape, src):
    """Add one Gaussian source to rows z in [z0, z1) of ``slab`` (which starts at z0)."""
    n3, n2, n1 = shape
    amp, (cx, cy, cz), (sx, sy, sz) = src
    lo = [max(0, int(math.floor(c - 4 * s))) for c, s in ((cx, sx), (cy, sy), (cz, sz))]
    hi = [min(n - 1, int(math.ceil(c + 4 * s))) for c, s, n in ((cx, sx, n1), (cy, sy, n2), (cz, sz, n3))]
    za, zb = max(lo[2], z0), min(hi[2], z1 - 1)
    if za > zb:
        return
    x = np.arange(lo[0], hi[0] + 1, dtype=np.float64)
    y = np.arange(lo[1], hi[1] + 1, dtype=np.float64)
    z = np.arange(za, zb + 1, dtype=np.float64)
    gx = np.exp(-0.5 * ((x - cx) / sx) ** 2)
    gy = np.exp(-0.5 * ((y - cy) / sy) ** 2)
    gz = np.exp(-0.5 * ((z - cz) / sz) ** 2)
    blob = amp * gz[:, None, None] * gy[None, :, None] * gx[None, None, :]
    view = slab[za - z0:zb - z0 + 1, lo[1]:hi[1] + 1, lo[0]:hi[0] + 1]
    view += blob.astype(np.float32)


def _band_rows(shape):
    """Per-x band centre and the y support (+-4 sigma) of the emission band."""
    n3, n2, n1 = shape
    sig = n2 / 64.0
    x = np.arange(n1, dtype=np.float64)
    y0 = n2 / 2.0 + (n2 / 8.0) * np.sin(2.0 * math.pi * x / n1)
    ylo = max(0, int(math.floor(y0.min() - 4 * sig)))
    yhi = min(n2 - 1, int(math.ceil(y0.max() + 4 * sig)))
    y = np.arange(ylo, yhi + 1, dtype=np.float64)
    g = 3.0 * np.exp(-0.5 * ((y[:, None] - y0[None, :]) / sig) ** 2)  # [ny][n1]
    return ylo, yhi, g


def cube(n1: int, n2: int, n3: int, seed: int, n_sources: int,
         sigma_range=(2.0, 6.0), band: bool = True, margin=None,
         nthreads: int | None = None, out: np.ndarray | None = None) -> np.ndarray:
    """Generate a ``[n3][n2][n1]`` float32 cube (see the module docstring)."""
    shape = (n3, n2, n1)
    if out is None:
        out = np.empty(shape, dtype=np.float32)
    assert out.shape == shape and out.dtype == np.float32 and out.flags.c_contiguous
    srng = np.random.Generator(np.random.PCG64([seed, 0x5EED]))
    sources = _source_params(srng, n_sources, shape, sigma_range, margin)
    if band:
        ylo, yhi, g = _band_rows(shape)
        zz = np.arange(n3, dtype=np.float64)
        ripple = 1.0 + 0.2 * np.cos(2.0 * math.pi * zz / (n3 / 4.0))
    slab_h = max(1, min(n3, (1 << 22) // max(1, n1 * n2) or 1))
    slabs = [(z0, min(n3, z0 + slab_h)) for z0 in range(0, n3, slab_h)]

    def work(idx):
        z0, z1 = slabs[idx]
        rng = np.random.Generator(np.random.PCG64([seed, idx]))
        sl = out[z0:z1]
        rng.standard_normal(out=sl, dtype=np.float32)
        if band:
            for z in range(z0, z1):
                sl[z - z0, ylo:yhi + 1, :] += (ripple[z] * g).astype(np.float32)
        for s in sources:
            _add_source_to_slab(sl, z0, z1, shape, s)

    nt = nthreads or threads()
    if nt == 1 or len(slabs) == 1:
        for i in range(len(slabs)):
            work(i)
    else:
        with ThreadPoolExecutor(nt) as ex:
            list(ex.map(work, range(len(slabs))))
    return out


# Named workloads (sizes from the benchmark configurations).
CONFIGS = {
    # 64^3, noise + 4 blobs elongated 3x along axis 3, one brick, 128^2, 2 views.
    "C1": dict(dims=(64, 64, 64), seed=1001, n_sources=4, sigma_range=(1.5, 3.0), band=False,
               margin=8.0, image=(128, 128)),
    # 512x512x1024 (1 GiB), noise + 200 sources + band, 2x2x2 bricks, 1024^2, 16 views.
    "C2": dict(dims=(512, 512, 1024), seed=1002, n_sources=200, band=True, image=(1024, 1024),
               bricks=(256, 256, 512), view_seed=2002, nviews=16),
    # 2048x2048x1536 (24 GiB), same generator, 256^3 bricks, 1024^2, 16 views.
    "C3": dict(dims=(2048, 2048, 1536), seed=1003, n_sources=4800, band=True, image=(1024, 1024),
               bricks=(256, 256, 256), view_seed=2003, nviews=16),
    # 64 requests (see batch_requests).
    "C4": dict(seed=1004, nreq=64),
    # 256x256x512 (128 MiB), 8 views at 512^2, differentiable.
    "C5": dict(dims=(256, 256, 512), seed=1005, n_sources=25, band=True, image=(512, 512),
               view_seed=2005, nviews=8, tf_seed=3005),
}


def config_sources(name: str) -> list:
    """The compact sources of a named cube: (amplitude, centre (x1, x2, x3), sigmas)."""
    c = CONFIGS[name]
    n1, n2, n3 = c["dims"]
    srng = np.random.Generator(np.random.PCG64([c["seed"], 0x5EED]))
    return _source_params(srng, c["n_sources"], (n3, n2, n1), c.get("sigma_range", (2.0, 6.0)), c.get("margin"))


def config_cube(name: str, nthreads: int | None = None, out=None) -> np.ndarray:
    c = CONFIGS[name]
    n1, n2, n3 = c["dims"]
    return cube(n1, n2, n3, c["seed"], c["n_sources"], c.get("sigma_range", (2.0, 6.0)),
                c.get("band", True), c.get("margin"), nthreads=nthreads, out=out)


def rot_axis(axis: int, deg: float) -> np.ndarray:
    """Right-handed rotation matrix about volume axis 1, 2 or 3 by ``deg`` degrees."""
    t = math.radians(deg)
    c, s = math.cos(t), math.sin(t)
    if axis == 1:
        return np.array([[1, 0, 0], [0, c, -s], [0, s, c]], dtype=np.float64)
    if axis == 2:
        return np.array([[c, 0, s], [0, 1, 0], [-s, 0, c]], dtype=np.float64)
    if axis == 3:
        return np.array([[c, -s, 0], [s, c, 0], [0, 0, 1]], dtype=np.float64)
    raise ValueError(axis)


def c1_views() -> list:
    """The two views of the 64^3 case: along axis 3, and 30 deg about axis 1 then 45 deg about axis 2."""
    return [np.eye(3), rot_axis(2, 45.0) @ rot_axis(1, 30.0)]


def random_rotation(rng) -> np.ndarray:
    """Uniform random rotation from a normalised quaternion of 4 seeded normals."""
    q = rng.standard_normal(4)
    w, x, y, z = q / np.linalg.norm(q)
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
        [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
        [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)],
    ], dtype=np.float64)


def random_views(n: int, seed: int) -> list:
    rng = np.random.Generator(np.random.PCG64(seed))
    return [random_rotation(rng) for _ in range(n)]


def tf_ramp(m: int = 256) -> np.ndarray:
    """Grey linear ramp: entry i has t = i/(m-1), RGB = (t, t, t), alpha = 0.02 t."""
    t = np.arange(m, dtype=np.float64) / (m - 1)
    return np.stack([t, t, t, 0.02 * t], axis=1).astype(np.float32)


def tf_colour(m: int = 256) -> np.ndarray:
    """Coloured ramp RGB = (t, 1 - t, 1/2), alpha = 0.02 t (catches channel mix-ups)."""
    t = np.arange(m, dtype=np.float64) / (m - 1)
    return np.stack([t, 1.0 - t, np.full_like(t, 0.5), 0.02 * t], axis=1).astype(np.float32)


def tf_noise_suppress(vmin: float, vmax: float, thresh: float = 6.0, amax: float = 0.2,
                      m: int = 256) -> np.ndarray:
    """Zero opacity below ``thresh`` (in data units), then a linear ramp to ``amax`` at vmax."""
    t = np.arange(m, dtype=np.float64) / (m - 1)
    v = vmin + t * (vmax - vmin)
    a = np.where(v < thresh, 0.0, amax * (v - thresh) / max(vmax - thresh, 1e-30))
    return np.stack([t, 0.5 + 0.5 * t, 1.0 - 0.5 * t, a], axis=1).astype(np.float32)


def _piecewise(rng, m, npts, lo, hi):
    xs = np.sort(rng.uniform(0.0, 1.0, npts))
    xs[0], xs[-1] = 0.0, 1.0
    ys = rng.uniform(lo, hi, npts)
    return np.interp(np.arange(m) / (m - 1), xs, ys)


def tf_random(rng, m: int = 256, npts: int = 8, amax: float = 0.05) -> np.ndarray:
    """Random piecewise-linear table with ``npts`` control points and alpha <= amax."""
    cols = [_piecewise(rng, m, npts, 0.0, 1.0) for _ in range(3)]
    cols.append(_piecewise(rng, m, npts, 0.0, amax))
    return np.stack(cols, axis=1).astype(np.float32)


def tf_perturbed(base: np.ndarray, seed: int) -> np.ndarray:
    """Smoothly perturbed copy: +0.05 smooth noise on RGB, x(1 + 0.2 smooth noise) on alpha."""
    rng = np.random.Generator(np.random.PCG64(seed))
    m = base.shape[0]
    out = base.astype(np.float64).copy()
    for ch in range(3):
        out[:, ch] += 0.05 * _piecewise(rng, m, 8, -1.0, 1.0)
    out[:, 3] *= 1.0 + 0.2 * _piecewise(rng, m, 8, -1.0, 1.0)
    return np.clip(out, 0.0, 1.0).astype(np.float32)


def batch_requests(seed: int = 1004, nreq: int = 64, dim_range=(32, 256), img_range=(64, 512)):
    """Descriptions of a batch of uneven render requests (volumes are generated lazily).

    Each request: dims ~U[dim_range] per axis (non-cubic), square image with side
    ~U[img_range], a random view and a random 8-point transfer function.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    reqs = []
    for i in range(nreq):
        dims = tuple(int(d) for d in rng.integers(dim_range[0], dim_range[1] + 1, 3))
        side = int(rng.integers(img_range[0], img_range[1] + 1))
        vol_seed = int(seed * 1000 + i)
        nsrc = max(2, int(round(200 * dims[0] * dims[1] * dims[2] / float(1 << 28))))
        reqs.append(dict(dims=dims, image=(side, side), view=random_rotation(rng),
                         tf=tf_random(rng), seed=vol_seed, n_sources=nsrc))
    return reqs
