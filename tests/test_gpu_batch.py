"""GPU checks of the batched persistent launch and of the autotuner (C ABI).

* one persistent, graph-replayed launch over uneven requests gives the same
  image bits as one plain render per request, on several replays with changed
  views, tables and outputs, with eager work and synchronisations between the
  replays (each replay compared with its own eager result);
* a shape change rebuilds the graph;
* parity of batched images with the FP64 oracle;
* the autotuner (render shapes and batch grid) returns a choice that keeps the
  images unchanged.
"""
import numpy as np
import pytest

import oracle
import paper_1008_0135_amd as vr
import synth
from gpu_util import parity

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu] {msg}", flush=True)


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = vr.vr_create(0)
    yield c
    vr.vr_destroy(c)


def _requests(seed, n, dim_range=(20, 72), img_range=(9, 90)):
    return synth.batch_requests(seed=seed, nreq=n, dim_range=dim_range, img_range=img_range)


def _volumes(ctx, descs):
    vols, arrays = [], []
    for d in descs:
        n1, n2, n3 = d["dims"]
        a = synth.cube(n1, n2, n3, seed=d["seed"], n_sources=d["n_sources"], sigma_range=(1.5, 3.0))
        arrays.append(a)
        vols.append(vr.vr_volume_create(ctx, a, (n1, n2, n3)))
    return vols, arrays


def _plain(ctx, vol, R, W, H, tf, vmin, vmax, params):
    vr.vr_tf_set(ctx, tf, vmin, vmax)
    out = torch.empty((1, H, W, 4), device="cuda")
    vr.vr_render(ctx, vol, [vr.make_view(R, W, H)], params, out)
    return out


def test_batch_replays_match_plain_renders(ctx):
    descs = _requests(71, 12)
    vols, arrays = _volumes(ctx, descs)
    params = vr.make_params(tau=0.99)
    cache = None
    rng = np.random.Generator(np.random.PCG64(72))
    for rep in range(3):
        _say(f"batch replay {rep}: 12 requests")
        outs, reqs, tfs, expect = [], [], [], []
        for i, d in enumerate(descs):
            W, H = d["image"]
            R = synth.random_rotation(rng) if rep else d["view"]
            tf = synth.tf_random(rng) if rep else d["tf"]
            mn, mx = float(arrays[i].min()), float(arrays[i].max())
            t = torch.from_numpy(tf).cuda()
            o = torch.full((H, W, 4), -3.0, device="cuda")
            tfs.append(t)
            outs.append(o)
            reqs.append(vr.make_request(vols[i], R, W, H, t, mn, mx, o))
            expect.append((R, W, H, tf, mn, mx))
        cache = vr.vr_render_batch(ctx, reqs, params, cache)
        torch.cuda.synchronize()
        got = [o.cpu().numpy() for o in outs]
        # eager renders between replays
        for i, (R, W, H, tf, mn, mx) in enumerate(expect):
            ref = _plain(ctx, vols[i], R, W, H, tf, mn, mx, params)
            torch.cuda.synchronize()
            assert np.array_equal(got[i], ref.cpu().numpy()[0]), (rep, i)
        if rep == 2:
            for i in (0, 5, 11):
                R, W, H, tf, mn, mx = expect[i]
                o = oracle.render(arrays[i], tf, [R], W, H, mn, mx, tau=0.99)
                parity(got[i][None], o, label=f"batch req {i}")
    vr.vr_batch_destroy(cache)
    for v in vols:
        vr.vr_volume_destroy(v)


def test_batch_shape_change_recaptures(ctx):
    _say("batch shape change")
    descs = _requests(73, 4)
    vols, arrays = _volumes(ctx, descs)
    params = vr.make_params(tau=2.0)
    cache = None
    for scale in (1, 2):
        outs, reqs = [], []
        for i, d in enumerate(descs):
            W, H = d["image"][0] * scale, d["image"][1]
            t = torch.from_numpy(d["tf"]).cuda()
            o = torch.empty((H, W, 4), device="cuda")
            outs.append((o, t))
            reqs.append(vr.make_request(vols[i], d["view"], W, H, t, 0.0, 0.0, o))
        cache = vr.vr_render_batch(ctx, reqs, params, cache)
        torch.cuda.synchronize()
        for i, d in enumerate(descs):
            W, H = d["image"][0] * scale, d["image"][1]
            mn, mx = float(arrays[i].min()), float(arrays[i].max())
            ref = _plain(ctx, vols[i], d["view"], W, H, d["tf"], mn, mx, params)
            torch.cuda.synchronize()
            assert np.array_equal(outs[i][0].cpu().numpy(), ref.cpu().numpy()[0])
    vr.vr_batch_destroy(cache)
    for v in vols:
        vr.vr_volume_destroy(v)


def test_autotune_keeps_images(ctx):
    _say("autotune render shapes and batch grid")
    vol = synth.cube(120, 100, 140, seed=74, n_sources=8, sigma_range=(2.0, 4.0))
    h = vr.vr_volume_create(ctx, vol, (120, 100, 140))
    vr.vr_volume_brick(h, vr.grid_spec((40, 50, 70)))
    tf = synth.tf_ramp(256)
    vr.vr_tf_set(ctx, tf)
    R = synth.random_views(1, 75)[0]
    view = vr.make_view(R, 200, 160)
    params = vr.make_params()
    out0 = torch.empty((1, 160, 200, 4), device="cuda")
    vr.vr_render(ctx, h, [view], params, out0)
    res = vr.vr_autotune(ctx, h, view, params)
    assert res.tile in (4, 8, 16) and res.ms > 0 and res.ms <= res.ms_default * 1.0001
    out1 = torch.empty_like(out0)
    vr.vr_render(ctx, h, [view], params, out1)
    torch.cuda.synchronize()
    assert np.array_equal(out0.cpu().numpy(), out1.cpu().numpy())
    descs = _requests(76, 6)
    vols, arrays = _volumes(ctx, descs)
    reqs, outs = [], []
    for i, d in enumerate(descs):
        W, H = d["image"]
        t = torch.from_numpy(d["tf"]).cuda()
        o = torch.empty((H, W, 4), device="cuda")
        outs.append((o, t))
        reqs.append(vr.make_request(vols[i], d["view"], W, H, t, 0.0, 0.0, o))
    r, cache = vr.vr_autotune_batch(ctx, reqs, params)
    assert r.waves_per_cu in (2, 4, 8, 16, 32)
    cache = vr.vr_render_batch(ctx, reqs, params, cache)
    torch.cuda.synchronize()
    for i, d in enumerate(descs):
        W, H = d["image"]
        mn, mx = float(arrays[i].min()), float(arrays[i].max())
        ref = _plain(ctx, vols[i], d["view"], W, H, d["tf"], mn, mx, params)
        torch.cuda.synchronize()
        assert np.array_equal(outs[i][0].cpu().numpy(), ref.cpu().numpy()[0])
    vr.vr_batch_destroy(cache)
    for v in vols + [h]:
        vr.vr_volume_destroy(v)


def test_c4_full_batch_parity(ctx):
    """The benchmark's batch at full size: 64 requests, volumes U[32, 256] per axis,
    images U[64, 512], random views and tables, after the batch autotuner.  Every
    request is checked against the FP64 oracle on strided rays (every 8th row and
    column) and against its own plain render bit for bit."""
    descs = synth.batch_requests(seed=synth.CONFIGS["C4"]["seed"], nreq=synth.CONFIGS["C4"]["nreq"])
    _say(f"C4 batch: generating {len(descs)} volumes")
    vols, arrays, reqs, outs, wins = [], [], [], [], []
    for d in descs:
        n1, n2, n3 = d["dims"]
        a = synth.cube(n1, n2, n3, seed=d["seed"], n_sources=d["n_sources"])
        arrays.append(a)
        vols.append(vr.vr_volume_create(ctx, a, (n1, n2, n3)))
        W, H = d["image"]
        t = torch.from_numpy(d["tf"]).cuda()
        o = torch.full((H, W, 4), -1.0, device="cuda")
        mn, mx = float(a.min()), float(a.max())
        outs.append((o, t))
        wins.append((mn, mx))
        reqs.append(vr.make_request(vols[-1], d["view"], W, H, t, mn, mx, o))
    params = vr.make_params(step=0.5, tau=0.99, ess=0)
    _say("C4 batch: autotune + render")
    r, cache = vr.vr_autotune_batch(ctx, reqs, params)
    cache = vr.vr_render_batch(ctx, reqs, params, cache)
    torch.cuda.synchronize()
    got = [o.cpu().numpy() for o, _ in outs]
    worst = 0.0
    for i, d in enumerate(descs):
        W, H = d["image"]
        mn, mx = wins[i]
        ref = _plain(ctx, vols[i], d["view"], W, H, d["tf"], mn, mx, params)
        torch.cuda.synchronize()
        assert np.array_equal(got[i], ref.cpu().numpy()[0]), f"request {i}: batch != plain render"
        yy, xx = np.meshgrid(np.arange(i % 8, H, 8), np.arange((3 * i) % 8, W, 8), indexing="ij")
        o = oracle.render_rays(arrays[i], d["tf"], [d["view"]], W, H, np.zeros(yy.size, np.int32), xx.ravel(),
                               yy.ravel(), mn, mx, tau=0.99)
        s = parity(got[i][yy.ravel(), xx.ravel()], o, label=f"C4 request {i} {d['dims']} {W}x{H}")
        worst = max(worst, s["worst"])
    _say(f"C4 batch: 64 requests match the oracle (worst {worst:.3g}) and their plain renders")
    vr.vr_batch_destroy(cache)
    for v in vols:
        vr.vr_volume_destroy(v)


@pytest.mark.parametrize("tile", [4, 16, 32])
def test_batch_tile_shapes_from_tune_cache(tile, tmp_path, monkeypatch):
    """Every tile shape the batch autotuner can choose (read back from a
    VR_TUNE_CACHE file, one entry per size class) gives the plain renders' bits."""
    _say(f"batch tile {tile} x {64 // tile} from the tune cache")
    descs = _requests(77, 10, dim_range=(24, 96), img_range=(17, 150))
    path = tmp_path / "tune.txt"
    # one entry per size class present (volume class floor(log2 voxels) / 3,
    # image class floor(log2 pixels) / 2, as the library documents)
    keys = set()
    for d in descs:
        n1, n2, n3 = d["dims"]
        W, H = d["image"]
        keys.add(f"batch/v{int(np.floor(np.log2(n1 * n2 * n3))) // 3}/i{int(np.floor(np.log2(W * H))) // 2}")
    path.write_text("".join(f"{k} {tile} 0 1 0.1\n" for k in sorted(keys)))
    monkeypatch.setenv("VR_TUNE_CACHE", str(path))
    c = vr.vr_create(0)
    try:
        vols, arrays = _volumes(c, descs)
        params = vr.make_params(tau=0.99)
        reqs, outs = [], []
        for i, d in enumerate(descs):
            W, H = d["image"]
            t = torch.from_numpy(d["tf"]).cuda()
            o = torch.full((H, W, 4), -2.0, device="cuda")
            outs.append((o, t))
            reqs.append(vr.make_request(vols[i], d["view"], W, H, t, 0.0, 0.0, o))
        assert vr.vr_batch_tiles(c, reqs) == [tile] * len(reqs)
        cache = vr.vr_render_batch(c, reqs, params, None)
        torch.cuda.synchronize()
        for i, d in enumerate(descs):
            W, H = d["image"]
            mn, mx = float(arrays[i].min()), float(arrays[i].max())
            ref = _plain(c, vols[i], d["view"], W, H, d["tf"], mn, mx, params)
            torch.cuda.synchronize()
            assert np.array_equal(outs[i][0].cpu().numpy(), ref.cpu().numpy()[0]), (tile, i)
        vr.vr_batch_destroy(cache)
        for v in vols:
            vr.vr_volume_destroy(v)
    finally:
        vr.vr_destroy(c)
