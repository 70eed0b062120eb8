"""Pins of the oracle's early-termination tie handling (paper Sec. 2.4: a ray
stops once its accumulated opacity reaches the threshold).

An FP32 renderer and the FP64 oracle can disagree on which sample is the first
with 1 - T >= tau when the opacity lands within rounding of tau; every stop in
that window is a correct result.  The oracle lists, for each flagged pixel,
every valid image (one per combination of valid stops of the pixel's
sub-volume chains).  These tests rebuild those images independently:

* axis-aligned rays through voxel columns, where the samples, the table lookup
  (``np.interp``) and the transmittance (``np.cumprod``) come from numpy, with
  the stop index chosen explicitly for every sample in the window;
* the same columns split into sub-volumes along axis 3, each with its own
  chain, combined with the over operator for every combination of stops;
* invariants on random views and partitions (the oracle's own image is among
  the candidates; candidate opacities sit in the window and grow with the stop).

Planted mistakes (a window one margin too wide or too narrow, a composite
without the front's transmittance, every candidate given the FP64 stop's
colour, transparent samples listed as extra images) are compiled into copies
of the oracle and each must fail a pin.
"""
import ctypes
import os
import subprocess

import numpy as np
import pytest

import oracle
import synth


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


# ------------------------------------------------------------- column model
def _column_samples(vol, tf, vmin, vmax):
    """Per-sample RGBA along every voxel column (R = I, pixel = column): [nk][n2][n1][4], z_k."""
    n3, n2, n1 = vol.shape
    M = tf.shape[0]
    nk = 2 * (n3 - 1)
    z = (np.arange(nk) + 0.5) * 0.5
    z0 = np.minimum(np.floor(z).astype(int), n3 - 2)
    f = z - z0
    col = vol.astype(np.float64)
    vals = (1 - f)[:, None, None] * col[z0] + f[:, None, None] * col[z0 + 1]
    s = np.clip((vals - vmin) / (vmax - vmin), 0, 1)
    u = s * (M - 1)
    rgba = np.stack([np.interp(u, np.arange(M), tf[:, c].astype(np.float64)) for c in range(4)], -1)
    return rgba, z


def _chain_states(rgba, tau, margin):
    """One chain (samples of one ray in one sub-volume, front first).

    Returns the list of valid (C, T) end states: the state after sample j for
    every j from the first sample with A >= tau - margin to the first with
    A >= tau + margin (or the last sample); a single state when A never
    reaches tau - margin (the end of the chain) or the window holds one stop.
    Also returns the state at the FP64 stop (first A >= tau).
    """
    a = rgba[:, 3]
    n = a.shape[0]
    if n == 0:
        return [(np.zeros(3), 1.0)], (np.zeros(3), 1.0)
    T = np.cumprod(1 - a)
    Tprev = np.concatenate([[1.0], T[:-1]])
    C = np.cumsum(Tprev[:, None] * a[:, None] * rgba[:, :3], axis=0)
    A = 1 - T
    reach = np.nonzero(A >= tau)[0]
    stop = int(reach[0]) if reach.size else n - 1
    lo = np.nonzero(A >= tau - margin)[0]
    if lo.size == 0:
        return [(C[-1], T[-1])], (C[-1], T[-1])
    hi = np.nonzero(A >= tau + margin)[0]
    last = int(hi[0]) if hi.size else n - 1
    # a sample of zero opacity leaves the state as it was: one image, listed once
    states = [(C[j], T[j]) for j in range(int(lo[0]), last + 1) if j == lo[0] or a[j] > 0]
    return states, (C[stop], T[stop])


def _over(states):
    Cs, A = np.zeros(3), 0.0
    for Cb, Tb in states:
        Cs = Cs + (1 - A) * Cb
        A = A + (1 - A) * (1 - Tb)
    return np.concatenate([Cs, [A]])


def _column_candidates(vol, tf, vmin, vmax, tau, margin, zcuts=()):
    """Per pixel: (oracle-style main image, list of valid images) from the column model.

    zcuts: interior faces along axis 3 (sub-volume k owns [cut_k, cut_{k+1}))."""
    rgba, z = _column_samples(vol, tf, vmin, vmax)
    n3, n2, n1 = vol.shape
    edges = [0.0, *zcuts, float(n3 - 1) + 1.0]
    out = {}
    for y in range(n2):
        for x in range(n1):
            chains, mains = [], []
            for b in range(len(edges) - 1):
                sel = (z >= edges[b]) & (z < edges[b + 1])
                if not sel.any():
                    continue
                st, main = _chain_states(rgba[sel, y, x], tau, margin)
                chains.append(st)
                mains.append(main)
            cands = [np.zeros(4)]
            combos = [[]]
            for st in chains:
                combos = [c + [s] for c in combos for s in st]
            cands = [_over(c) for c in combos]
            out[(y, x)] = (_over(mains), cands)
    return out


def _column_case(seed, n1=6, n2=5, n3=48, zero_low=False):
    rng = _rng(seed)
    vol = rng.normal(0, 1, (n3, n2, n1)).astype(np.float32)
    tf = synth.tf_colour(16)
    tf[:, 3] = np.linspace(0.02, 0.2, 16, dtype=np.float32)
    if zero_low:  # runs of transparent samples (values in the lower half)
        tf[:8, 3] = 0.0
        tf[8:, 3] = np.linspace(0.05, 0.5, 8, dtype=np.float32)
    return vol, tf, float(vol.min()), float(vol.max())


def _check_columns(orc, tau, margin, zcuts=(), seed=1, zero_low=False):
    """The oracle's valid images of every column pixel equal the column model's."""
    vol, tf, vmin, vmax = _column_case(seed, n1=10, n2=9, zero_low=zero_low) if zero_low else _column_case(seed)
    n3, n2, n1 = vol.shape
    bricks = None
    if zcuts:
        edges = [0, *zcuts, n3 - 1]
        bricks = [((0, 0, edges[k]), (n1 - 1, n2 - 1, edges[k + 1]), (1, 1, 1 if k == len(edges) - 2 else 0))
                  for k in range(len(edges) - 1)]
    res = orc.render(vol, tf, [np.eye(3)], n1, n2, vmin, vmax, tau=tau, extent=float(n1), bricks=bricks,
                     ert_margin=margin)
    want = _column_candidates(vol, tf, vmin, vmax, tau, margin, zcuts)
    flags = res["flags"][0]
    # interior columns are clear of the box faces (the border ones lie on them)
    assert ((flags[1:-1, 1:-1] & orc.FLAG_GEOM) == 0).all()
    t = res["ties"]
    pos = {int(i): j for j, i in enumerate(t["index"])}
    nties = 0
    for (y, x), (main, cands) in want.items():
        if flags[y, x] & orc.FLAG_GEOM:
            continue  # a border ray on a box face: hit or miss are both correct
        np.testing.assert_allclose(res["image"][0][y, x], main, rtol=0, atol=1e-12)
        q = y * n1 + x
        if len(cands) == 1:
            assert not flags[y, x] & orc.FLAG_ERT, (y, x)
            continue
        nties += 1
        assert flags[y, x] & orc.FLAG_ERT, (y, x)
        j = pos[q]
        got = t["cand"][j][:t["ncand"][j]]
        assert got.shape[0] == len(cands), ((y, x), got.shape[0], len(cands))
        # same set: every expected image is listed, and nothing else
        for c in cands:
            assert np.abs(got - c).max(axis=1).min() <= 1e-12, ((y, x), c)
        for g in got:
            assert min(np.abs(g - c).max() for c in cands) <= 1e-12, ((y, x), g)
    return nties


@pytest.mark.parametrize("tau,margin", [(0.9, 3e-3), (0.99, 1e-3), (0.8, 1e-2)])
def test_whole_column_candidates(orc, tau, margin):
    """Whole volume: the valid images are exactly stop-at-j for j in the window."""
    assert _check_columns(orc, tau, margin) >= 5


def test_transparent_samples_in_window(orc):
    """Zero-opacity samples inside a tie window repeat the previous image: each valid
    image is listed once (a window spanning a long transparent run stays listable)."""
    assert _check_columns(orc, 0.6, 2e-2, zero_low=True) >= 3
    assert _check_columns(orc, 0.5, 3e-2, (20,), zero_low=True) >= 3


@pytest.mark.parametrize("zcuts", [(20,), (10, 31)])
def test_bricked_column_candidates(orc, zcuts):
    """Sub-volumes along the ray: every combination of the chains' valid stops, composited."""
    assert _check_columns(orc, 0.5, 2e-2, zcuts) >= 5


def test_default_margin_exact_tie(orc):
    """tau set to a pixel's own FP64 opacity after some sample: that pixel is a tie with
    the default margin, and its stop-one-earlier / at / later images are listed."""
    vol, tf, vmin, vmax = _column_case(3)
    rgba, _ = _column_samples(vol, tf, vmin, vmax)
    T = np.cumprod(1 - rgba[..., 3], axis=0)
    y, x, k = 2, 3, 17
    tau = float(1 - T[k, y, x])
    res = orc.render(vol, tf, [np.eye(3)], vol.shape[2], vol.shape[1], vmin, vmax, tau=tau,
                     extent=float(vol.shape[2]))
    assert res["flags"][0][y, x] & orc.FLAG_ERT
    want = _column_candidates(vol, tf, vmin, vmax, tau, 1e-5)[(y, x)][1]
    j = list(res["ties"]["index"]).index(y * vol.shape[2] + x)
    got = res["ties"]["cand"][j][:res["ties"]["ncand"][j]]
    assert len(want) >= 2 and got.shape[0] == len(want)
    for c in want:
        assert np.abs(got - c).max(axis=1).min() <= 1e-12


def test_candidate_invariants_random_views(orc):
    """Random views, grid and longest-axis partitions, wide margin: the oracle's image is
    one of the listed ones; whole-volume candidates have A >= tau - m, all but the
    last A < tau + m, and A grows with the stop."""
    rng = _rng(5)
    vol = synth.cube(20, 18, 24, seed=5, n_sources=6, sigma_range=(1.5, 3.0))
    tf = synth.tf_colour(32)
    tf[:, 3] = np.linspace(0.04, 0.3, 32, dtype=np.float32)
    vmin, vmax = float(vol.min()), float(vol.max())
    views = synth.random_views(2, 6)
    tau, m = 0.9, 2e-3
    for bricks in (None, {"grid": (8, 8, 12)}, {"boxes": oracle.kd_boxes((20, 18, 24), 5)}):
        res = orc.render(vol, tf, views, 40, 36, vmin, vmax, tau=tau, bricks=bricks, ert_margin=m)
        t = res["ties"]
        assert t["index"].size > 20
        assert (t["ncand"] >= 2).all()
        img = res["image"].reshape(-1, 4)
        for j, q in enumerate(t["index"]):
            c = t["cand"][j][:t["ncand"][j]]
            assert np.abs(c - img[q]).max(axis=1).min() <= 1e-15
            if bricks is None:
                A = c[:, 3]
                assert (A >= tau - m - 1e-15).all()
                assert (A[:-1] < tau + m).all()
                assert (np.diff(A) > 0).all()
    del rng


def test_match_error(orc):
    """match_error takes the closest listed image, all four channels together."""
    vol, tf, vmin, vmax = _column_case(4)
    res = orc.render(vol, tf, [np.eye(3)], vol.shape[2], vol.shape[1], vmin, vmax, tau=0.9,
                     extent=float(vol.shape[2]), ert_margin=3e-3)
    t = res["ties"]
    j = int(np.argmax(t["ncand"]))
    q = int(t["index"][j])
    got = res["image"].copy().reshape(-1, 4)
    got[q] = t["cand"][j][t["ncand"][j] - 1]  # the latest valid stop
    e = orc.match_error(got.reshape(res["image"].shape), res)
    assert e.reshape(-1)[q] == 0.0 and e.max() == 0.0
    # channels from two different candidates do not match any one of them
    mix = t["cand"][j][0].copy()
    mix[3] = t["cand"][j][t["ncand"][j] - 1][3]
    got[q] = mix
    e = orc.match_error(got.reshape(res["image"].shape), res)
    assert e.reshape(-1)[q] > 1e-6


# ------------------------------------------------------------ planted mistakes
_MUTANTS = {
    "window one margin too wide": (
        "if (A >= sc->tau + sc->ert_margin) ch->hi_seen = 1;",
        "if (A >= sc->tau + 2.0 * sc->ert_margin) ch->hi_seen = 1;"),
    "stop-one-earlier dropped": (
        "if (A >= sc->tau - sc->ert_margin) ch->lo_seen = 1;",
        "if (A >= sc->tau) ch->lo_seen = 1;"),
    "composite without the front's transmittance": (
        "for (int c = 0; c < 3; c++) C[c] = C[c] + (1.0 - A) * Cb[c];",
        "for (int c = 0; c < 3; c++) C[c] = C[c] + Cb[c];"),
    "transparent samples listed again": (
        "if (ch->lo_seen && (ch->nst == 0 || a > 0.0)) {",
        "if (ch->lo_seen) {"),
    "candidates keep the FP64 stop's colour": (
        "for (int c = 0; c < 3; c++) C[c] = ch->stC[j][c];",
        "for (int c = 0; c < 3; c++) C[c] = ch->C[c];"),
}


@pytest.mark.parametrize("name", sorted(_MUTANTS))
def test_planted_mistakes_fail(orc, name, tmp_path):
    src = open(os.path.join(os.path.dirname(oracle.__file__), "vr_oracle.c")).read()
    old, new = _MUTANTS[name]
    assert src.count(old) == 1, name
    path = tmp_path / "mut.c"
    path.write_text(src.replace(old, new))
    so = str(tmp_path / "libmut.so")
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=c11", "-o", so, str(path), "-lm"])
    saved = oracle._lib
    oracle._lib = oracle._bind(ctypes.CDLL(so))
    try:
        failed = False
        for args in ((0.9, 3e-3, ()), (0.5, 2e-2, (10, 31)), (0.6, 2e-2, (), 1, True)):
            try:
                _check_columns(oracle, *args)
            except AssertionError:
                failed = True
        assert failed, f"planted mistake not caught: {name}"
    finally:
        oracle._lib = saved
