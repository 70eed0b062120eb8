"""Benchmark: bricked ray casting + sort-last compositing on one MI355X.

Default workload: a 2048 x 2048 x 1536 float32 cube (24 GiB; noise + 4800
elongated sources + emission band), 256^3 bricks with 1-voxel ghosts and
per-brick ranges, 1024 x 1024 orthographic frames, 16 seeded random views,
step 0.5 voxel, grey ramp transfer function (alpha = 0.02 t), early
termination at opacity 0.99 (per brick, sort-last).  The cube is also kept as
a permuted copy (axes 2, 3, 1; built before timing) from which the views
looking mostly along axis 1 are rendered.  One step renders the 16 views
(march + composite per view) through the C ABI.  Further legs on the same
cube and views: perspective projection, maximum intensity projection, early
termination over the whole ray; then a 64-request batched launch and a
forward + backward pass of the differentiable path.

Prints one JSON line: Gsamples/s (nominal lattice samples per second), ms per
step and per frame, the march kernel's HBM roofline fraction (algorithmic
bytes per launch / average launch time, from HIP events recorded on the
launch stream), and the FP64 oracle timed on this host on a bounded ray
sample of the same workload (which also gives a parity figure).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import paper_1008_0135_amd as vr  # noqa: E402
import synth  # noqa: E402

METRIC = "Gsamples/s + ms per 1024² frame (fwd, batched, fwd+bwd), % of HBM roofline"
HBM_PEAK_GBS = 8000.0
# non-packed FP32 vector issue: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz, lane-ops/s
VALU_PEAK_LANE_OPS = 256 * 4 * 16 * 2.4e9
# algorithmic VALU work of one sample (trilinear 7 lerps = 14, normalisation 3,
# table lerp of four channels 8, compositing about 9, position and index
# arithmetic about 16): an estimate of the lane operations a sample needs
LANE_OPS_PER_SAMPLE = 50


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def threads_used():
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1


def _events_ms(fn, reps, stream):
    import torch
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    fn()
    torch.cuda.synchronize()
    a.record(stream)
    for _ in range(reps):
        fn()
    b.record(stream)
    b.synchronize()
    return a.elapsed_time(b) / reps


def stream_peak(stream, gib=4.0):
    """Measured stream peak: a device-to-device copy of `gib` GiB (reads + writes
    counted), timed with HIP events on the launch stream."""
    import torch
    n = int(gib * 2**30) // 4
    x = torch.ones(n, device="cuda")
    y = torch.empty_like(x)
    ms = _events_ms(lambda: y.copy_(x), 5, stream)
    del x, y
    torch.cuda.empty_cache()
    return 2.0 * n * 4 / (ms * 1e-3) / 1e9


def mc_transparent(mm, tf, vmin, vmax):
    """Per macrocell: every table entry its range can reach (one entry of margin
    each side) has opacity 0, as for bricks."""
    M = tf.shape[0]
    scale = (M - 1) / (vmax - vmin) if vmax > vmin else 0.0
    u0 = np.clip((mm[..., 0].astype(np.float64) - vmin) * scale, 0, M - 1)
    u1 = np.clip((mm[..., 1].astype(np.float64) - vmin) * scale, 0, M - 1)
    i0 = np.maximum(0, np.floor(u0).astype(np.int64) - 1)
    i1 = np.minimum(M - 1, np.ceil(u1).astype(np.int64) + 1)
    nz = np.concatenate([[0], np.cumsum(tf[:, 3] != 0)])  # entries with opacity != 0 before index i
    return (nz[i1 + 1] - nz[i0]) == 0


def bench_tf_suppress(ctx, h, dims, views_R, W, H, vmin, vmax, stream):
    """The same cube and views with the noise-suppressing table (opacity 0 below
    6 sigma): whole bricks and macrocell steps whose range is transparent are
    skipped.  Algorithmic bytes: the voxels of the macrocells that may be
    opaque (each read once) + the brick-image writes."""
    import torch
    tf = synth.tf_noise_suppress(vmin, vmax, thresh=6.0)
    vr.vr_tf_set(ctx, tf)
    views = [vr.make_view(R, W, H) for R in views_R]
    params = vr.make_params(step=0.5, tau=0.99, ess=1)
    out = torch.empty((len(views), H, W, 4), device="cuda")
    ms = _events_ms(lambda: vr.vr_render(ctx, h, views, params, out, stream), 3, stream)
    vr.vr_set_profiling(ctx, True)
    vr.vr_render(ctx, h, views, params, out, stream)
    t, c = vr.vr_stage_times(ctx)
    vr.vr_set_profiling(ctx, False)
    march = t[vr.VR_STAGE_MARCH] / max(1, c[vr.VR_STAGE_MARCH])
    edge, cnt, mm = vr.vr_volume_macrocell_info(h)
    clear = mc_transparent(mm, tf, vmin, vmax)
    n = np.array(dims, np.int64)
    # voxels per macrocell (the last along each axis may be shorter)
    ext = [np.minimum(edge, (n[i] - 1) - edge * np.arange(cnt[i])) for i in range(3)]
    vox = ext[2][:, None, None] * ext[1][None, :, None] * ext[0][None, None, :]
    alg = float(4 * vox[~clear].sum())
    log(f"tf_suppress: {ms / len(views):.3f} ms/frame, march {march:.3f} ms/launch, "
        f"{clear.mean() * 100:.2f} % of macrocells transparent")
    vr.vr_tf_set(ctx, synth.tf_ramp(256))
    return {"workload": "same cube and views, noise-suppressing table (opacity 0 below 6 sigma, ramp to 0.2), "
                        "16^3 macrocells, bricks and macrocell steps of zero opacity skipped",
            "ms_per_frame": round(ms / len(views), 4), "march_ms_per_launch": round(march, 4),
            "macrocells_skipped_frac": round(float(clear.mean()), 5),
            "roofline": {"bound": "hbm", "achieved": round(alg / (march * 1e-3) / 1e9, 1), "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": round(alg / (march * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                         "alg_bytes_per_launch": int(alg),
                         "alg_bytes": "voxels of the macrocells that may be opaque x 4 B (brick images excluded)"}}


def bench_c2(ctx, stream):
    """512 x 512 x 1024 (1 GiB) in 2 x 2 x 2 bricks, 16 views at 1024^2, ramp
    table, per-brick termination: more than one sample per voxel, so the VALU
    and HBM fractions are both reported."""
    import torch
    cfg = synth.CONFIGS["C2"]
    n1, n2, n3 = cfg["dims"]
    W, H = cfg["image"]
    vol = synth.config_cube("C2")
    h = vr.vr_volume_create(ctx, vol, (n1, n2, n3), on_device=False)
    vr.vr_volume_brick(h, vr.grid_spec(cfg["bricks"]))
    bricks = vr.vr_volume_brick_info(h)
    vr.vr_tf_set(ctx, synth.tf_ramp(256))
    views = [vr.make_view(R, W, H) for R in synth.random_views(cfg["nviews"], cfg["view_seed"])]
    params = vr.make_params(step=0.5, tau=0.99, ess=1)
    nominal = sum(vr.vr_count_samples((n1, n2, n3), v, 0.5) for v in views)
    out = torch.empty((len(views), H, W, 4), device="cuda")
    ms = _events_ms(lambda: vr.vr_render(ctx, h, views, params, out, stream), 3, stream)
    vr.vr_set_profiling(ctx, True)
    vr.vr_render(ctx, h, views, params, out, stream)
    t, c = vr.vr_stage_times(ctx)
    vr.vr_set_profiling(ctx, False)
    march = t[vr.VR_STAGE_MARCH] / max(1, c[vr.VR_STAGE_MARCH])
    spec = vr.grid_spec(cfg["bricks"])
    alg = 0.0
    for v in views:
        rects, _ = vr.vr_plan_view((n1, n2, n3), spec, v)
        for b, (x0, y0, w, hh) in enumerate(rects):
            if w and hh:
                d = bricks[b]
                vx = 1
                for i in range(3):
                    vx *= (d.hi[i] - d.lo[i] + (1 if d.closed[i] else 0))
                alg += 4 * vx + 16 * w * hh
    alg /= len(views)
    per_launch = nominal / len(views)
    vr.vr_volume_destroy(h)
    gsps = nominal / ms / 1e6
    log(f"C2: {ms / len(views):.3f} ms/frame, {gsps:.1f} Gsamples/s, march {march:.3f} ms/launch")
    return {"workload": f"{n1}x{n2}x{n3} f32 cube (1 GiB), 2x2x2 bricks, {W}x{H}, {len(views)} views, ramp table, "
                        "tau 0.99 per brick", "ms_per_frame": round(ms / len(views), 4),
            "gsamples_per_s": round(gsps, 3), "march_ms_per_launch": round(march, 4),
            "roofline_hbm": {"achieved": round(alg / (march * 1e-3) / 1e9, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                             "frac": round(alg / (march * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                             "alg_bytes_per_launch": int(alg)},
            "roofline_valu": {"achieved": round(LANE_OPS_PER_SAMPLE * per_launch / (march * 1e-3) / 1e12, 2),
                              "peak": round(VALU_PEAK_LANE_OPS / 1e12, 2), "unit": "T lane-ops/s",
                              "frac": round(LANE_OPS_PER_SAMPLE * per_launch / (march * 1e-3) / VALU_PEAK_LANE_OPS, 4),
                              "lane_ops_per_sample": LANE_OPS_PER_SAMPLE}}


def bench_batched(ctx, stream):
    """64 uneven requests: one persistent graph-replayed launch vs 64 plain renders."""
    import torch
    t0 = time.time()
    descs = synth.batch_requests(seed=synth.CONFIGS["C4"]["seed"], nreq=synth.CONFIGS["C4"]["nreq"])
    vols, reqs, plain = [], [], []
    nominal = 0
    for d in descs:
        n1, n2, n3 = d["dims"]
        a = synth.cube(n1, n2, n3, seed=d["seed"], n_sources=d["n_sources"])
        h = vr.vr_volume_create(ctx, a, (n1, n2, n3), on_device=False)
        vols.append(h)
        W, H = d["image"]
        tf = torch.from_numpy(d["tf"]).cuda()
        out = torch.empty((H, W, 4), device="cuda")
        mn, mx = float(a.min()), float(a.max())
        view = vr.make_view(d["view"], W, H)
        nominal += vr.vr_count_samples((n1, n2, n3), view, 0.5)
        reqs.append(vr.make_request(h, d["view"], W, H, tf, mn, mx, out))
        plain.append((h, view, d["tf"], mn, mx, out[None], tf))
    log(f"batched: 64 requests generated and uploaded in {time.time() - t0:.1f} s, {nominal:.3g} samples")
    params = vr.make_params(step=0.5, tau=0.99, ess=0)
    tune, cache = vr.vr_autotune_batch(ctx, reqs, params, None, stream)

    def run_batch():
        vr.vr_render_batch(ctx, reqs, params, cache, stream)

    def run_plain():
        for h, view, tf, mn, mx, out, _ in plain:
            vr.vr_tf_set(ctx, tf, mn, mx, stream)
            vr.vr_render(ctx, h, [view], params, out, stream)

    ms_b = _events_ms(run_batch, 10, stream)
    ms_p = _events_ms(run_plain, 3, stream)
    tiles = vr.vr_batch_tiles(ctx, reqs)
    vr.vr_batch_destroy(cache)
    vbytes = 0
    for h in vols:
        vr.vr_volume_destroy(h)
    for d in descs:
        vbytes += 4 * d["dims"][0] * d["dims"][1] * d["dims"][2] + 16 * d["image"][0] * d["image"][1]
    # the same 64 requests as plain launches with the batch's shapes: the gather
    # march with each request's tuned tile (32 x 2 tiles run as 16 x 4, the
    # widest the plain gather takes)
    import os as _os
    _os.environ["VR_MARCH"] = "gather"
    ctx_g = vr.vr_create(0)
    del _os.environ["VR_MARCH"]
    same = []
    for i, d in enumerate(descs):
        n1, n2, n3 = d["dims"]
        a = synth.cube(n1, n2, n3, seed=d["seed"], n_sources=d["n_sources"])
        hg = vr.vr_volume_create(ctx_g, a, (n1, n2, n3), on_device=False)
        _, view, tf, mn, mx, out, _ = plain[i]
        same.append((hg, view, tf, mn, mx, out, vr.make_params(step=0.5, tau=0.99, ess=0, tile=min(16, tiles[i]))))

    def run_same():
        for hg, view, tf, mn, mx, out, pp in same:
            vr.vr_tf_set(ctx_g, tf, mn, mx, stream)
            vr.vr_render(ctx_g, hg, [view], pp, out, stream)

    ms_s = _events_ms(run_same, 3, stream)
    for hg, *_ in same:
        vr.vr_volume_destroy(hg)
    vr.vr_destroy(ctx_g)
    ops = LANE_OPS_PER_SAMPLE * nominal
    log(f"batched: {ms_b:.3f} ms per 64-request batch ({nominal / ms_b / 1e6:.1f} Gsamples/s), "
        f"64 plain launches {ms_p:.3f} ms (same shapes: {ms_s:.3f} ms), grid {tune.waves_per_cu} waves/CU, "
        f"tiles {dict((t, tiles.count(t)) for t in sorted(set(tiles)))}")
    return {"workload": "64 requests, volumes U[32,256]^3 (non-cubic), images U[64,512]^2, random views and "
                        "8-point tables, one persistent hipGraph launch; tile shape per size class and grid "
                        "from the autotuner", "ms_per_batch": round(ms_b, 4),
            "gsamples_per_s": round(nominal / ms_b / 1e6, 3), "ms_64_plain_launches": round(ms_p, 4),
            "speedup_vs_plain": round(ms_p / ms_b, 3),
            "ms_64_plain_launches_same_shapes": round(ms_s, 4),
            "speedup_vs_plain_same_shapes": round(ms_s / ms_b, 3), "nominal_samples": int(nominal),
            "waves_per_cu": tune.waves_per_cu,
            "tiles": {f"{t}x{64 // t}": tiles.count(t) for t in sorted(set(tiles))},
            "roofline": {"bound": "alu", "achieved": round(ops / (ms_b * 1e-3) / 1e12, 2),
                         "peak": round(VALU_PEAK_LANE_OPS / 1e12, 2), "unit": "T lane-ops/s",
                         "frac": round(ops / (ms_b * 1e-3) / VALU_PEAK_LANE_OPS, 4),
                         "lane_ops_per_sample": LANE_OPS_PER_SAMPLE,
                         "hbm_frac": round(vbytes / (ms_b * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}}


def bench_fwd_bwd(ctx, stream):
    """256x256x512, 8 views at 512^2: forward with checkpoints + adjoint (L2 loss to a perturbed-table target)."""
    import torch
    c = synth.CONFIGS["C5"]
    n1, n2, n3 = c["dims"]
    W, H = c["image"]
    a = synth.config_cube("C5")
    dvol = torch.from_numpy(a).cuda()
    h = vr.vr_volume_wrap(ctx, dvol, (n1, n2, n3), stream)
    vmin, vmax = float(a.min()) - 0.5, float(a.max()) + 0.5
    views = [vr.make_view(R, W, H) for R in synth.random_views(c["nviews"], c["view_seed"])]
    nominal = sum(vr.vr_count_samples((n1, n2, n3), v, 0.5) for v in views)
    tf = synth.tf_colour(256)
    target_tf = synth.tf_perturbed(tf, c["tf_seed"])
    params = vr.make_params(step=0.5, tau=2.0, ess=0, ckpt_K=32)
    target = torch.empty((len(views), H, W, 4), device="cuda")
    vr.vr_tf_set(ctx, target_tf, vmin, vmax, stream)
    vr.vr_render(ctx, h, views, params, target, stream)
    vr.vr_tf_set(ctx, tf, vmin, vmax, stream)
    out = torch.empty_like(target)
    gtf = torch.empty((256, 4), device="cuda")
    gvol = torch.empty_like(dvol)

    def fwd():
        vr.vr_render(ctx, h, views, params, out, stream)

    def fwd_bwd():
        st = vr.vr_render(ctx, h, views, params, out, stream, save=True)
        g = out - target
        vr.vr_render_backward(ctx, h, st, g, gtf, gvol, False, stream)
        vr.vr_state_destroy(st)

    ms_f = _events_ms(fwd, 5, stream)
    ms_fb = _events_ms(fwd_bwd, 3, stream)
    # checkpoint interval the plan took per view (ckpt_K = 32 bounds it)
    st = vr.vr_render(ctx, h, views, params, out, stream, save=True)
    spg = [vr.vr_state_info(st, i)[2] for i in range(len(views))]
    lay = [vr.vr_state_info(st, i)[1] for i in range(len(views))]
    # kernel time of the backward alone (stage timer on the launch stream)
    vr.vr_set_profiling(ctx, True)
    vr.vr_render_backward(ctx, h, st, out - target, gtf, gvol, False, stream)
    tt, _ = vr.vr_stage_times(ctx)
    vr.vr_set_profiling(ctx, False)
    vr.vr_state_destroy(st)
    ms_b_kernels = tt[vr.VR_STAGE_BACKWARD]
    vr.vr_volume_destroy(h)
    log(f"fwd+bwd: forward {ms_f:.3f} ms, forward+backward {ms_fb:.3f} ms for {len(views)} views of 512^2 "
        f"(backward kernels {ms_b_kernels:.3f} ms; checkpoints every {min(spg):.1f}-{max(spg):.1f} samples)")
    return {"workload": "256x256x512 f32 cube, 8 views at 512x512, colour-ramp table, L2 loss against a "
                        "perturbed-table target, ckpt_K 32 (checkpoint groups of at most 3 cell layers on the "
                        "ring layout), gradients to table and voxels",
            "ms_forward": round(ms_f, 4), "ms_forward_backward": round(ms_fb, 4),
            "ms_backward_kernels": round(ms_b_kernels, 4),
            "gsamples_per_s_forward": round(nominal / ms_f / 1e6, 3),
            "gsamples_per_s_forward_backward": round(nominal / ms_fb / 1e6, 3),
            "backward_over_forward": round((ms_fb - ms_f) / ms_f, 3), "nominal_samples": int(nominal),
            "samples_per_checkpoint": {"min": round(min(spg), 2), "max": round(max(spg), 2)},
            "cell_layers_per_group": sorted(set(lay))}


def bench_variants(ctx, h, dims, views_R, W, H, stream, plan=None):
    """The same cube and views rendered with a perspective camera (eye at twice
    the half diagonal from the centre: a 53-degree field of view at the
    box-diagonal extent), as a maximum intensity projection, and with the
    opacity test over the whole ray (bricks in front-to-back waves).  plan =
    (brick size, brick records, table, vmin, vmax): the perspective leg then
    also reports its march's HBM roofline fraction."""
    import torch
    n = np.array(dims, np.float64)
    eye = float(np.sqrt(((n - 1) ** 2).sum()))  # 2 x half diagonal
    out = torch.empty((len(views_R), H, W, 4), device="cuda")
    res = {}
    for name, mode, ed, scope in (("perspective", 0, eye, 0), ("mip", vr.VR_MODE_MIP, 0.0, 0),
                                  ("global_ert", 0, 0.0, vr.VR_ERT_GLOBAL)):
        views = [vr.make_view(R, W, H, eye_dist=ed) for R in views_R]
        params = vr.make_params(step=0.5, tau=0.99, ess=1, mode=mode, ert_scope=scope)
        nominal = sum(vr.vr_count_samples(dims, v, 0.5) for v in views)
        ms = _events_ms(lambda: vr.vr_render(ctx, h, views, params, out, stream), 3, stream)
        log(f"{name}: {ms / len(views):.3f} ms/frame, {nominal / ms / 1e6:.1f} Gsamples/s")
        res[name] = {"ms_per_frame": round(ms / len(views), 4), "gsamples_per_s": round(nominal / ms / 1e6, 3),
                     "nominal_samples_per_frame": int(nominal // len(views))}
        if name == "perspective" and plan is not None:
            # the march stage of one call (all its launches), per view
            vr.vr_set_profiling(ctx, True)
            vr.vr_render(ctx, h, views, params, out, stream)
            st, _ = vr.vr_stage_times(ctx)
            vr.vr_set_profiling(ctx, False)
            march = st[vr.VR_STAGE_MARCH] / len(views)
            alg = float(np.mean([b + i for b, i, _ in alg_bytes_per_view(dims, plan[0], plan[1], views, *plan[2:])]))
            ach = alg / (march * 1e-3) / 1e9
            res[name]["march_ms_per_view"] = round(march, 4)
            res[name]["roofline"] = {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                     "frac": round(ach / HBM_PEAK_GBS, 4), "alg_bytes_per_launch": int(alg),
                                     "alg_bytes": "interior voxels of the marched bricks x 4 B + brick images x 16 B"}
    res["perspective"]["eye_dist"] = round(eye, 2)
    return res


def alg_bytes_per_view(dims, brick_size, bricks, views, tf, vmin, vmax):
    """Per view (brick bytes, image bytes, bricks): the interior voxels of the
    bricks the renderer marches (non-empty rectangle, not transparent under the
    table) x 4 B and their brick images x 16 B, from the host plan (the same
    rectangles and the same transparent-brick test as the renderer)."""
    spec = vr.grid_spec(brick_size)
    res = []
    for v in views:
        rects, _ = vr.vr_plan_view(dims, spec, v)
        brick_bytes = 0
        img_bytes = 0
        count = 0
        for b, (x0, y0, w, hh) in enumerate(rects):
            d = bricks[b]
            if w == 0 or hh == 0 or brick_transparent(d.vmin, d.vmax, tf, vmin, vmax):
                continue
            vox = 1
            for i in range(3):
                vox *= (d.hi[i] - d.lo[i] + (1 if d.closed[i] else 0))
            brick_bytes += 4 * vox
            img_bytes += 16 * w * hh
            count += 1
        res.append((brick_bytes, img_bytes, count))
    return res


def brick_transparent(bmin, bmax, tf, vmin, vmax):
    """A brick is skipped when every table entry its value range can reach
    (one entry of margin each side) has opacity 0."""
    M = tf.shape[0]

    def u(x):
        t = (x - vmin) / (vmax - vmin) if vmax > vmin else 0.0
        return min(1.0, max(0.0, t)) * (M - 1)

    i0 = max(0, int(np.floor(u(bmin))) - 1)
    i1 = min(M - 1, int(np.ceil(u(bmax))) + 1)
    return bool((tf[i0:i1 + 1, 3] == 0).all())


def traffic_model(config, twin):
    """Bytes the footprint-cell march's window loads request per launch on the
    config's views, from the host plan (vr_plan_cells; no GPU): the rendered
    bricks' own voxels, the line-granular union of the windows (ghost layers
    and the rows two bricks' windows share), the sum of the windows (halo
    shared by neighbouring cells), the same in 64-byte segments and in 128-byte
    lines (partly used lines)."""
    cfg = synth.CONFIGS[config]
    W, H = cfg["image"]
    spec = vr.grid_spec(cfg["bricks"], twin=twin)
    keys = ["own_bytes", "union_bytes", "window_bytes", "segment_bytes", "line_bytes"]
    tot = {k: 0.0 for k in keys}
    views = synth.random_views(cfg["nviews"], cfg["view_seed"])
    for R in views:
        t = vr.vr_plan_cells(cfg["dims"], spec, vr.make_view(R, W, H))
        for k in keys:
            tot[k] += getattr(t, k)
    n = len(views)
    return {"workload": config, "views": n, "per_launch_gb": {k[:-6]: round(tot[k] / n / 1e9, 3) for k in keys},
            "over_own": {k[:-6]: round(tot[k] / tot["own_bytes"], 4) for k in keys}}


def counter_traffic(config):
    """HBM bytes per march launch from the committed rocprofv3 counter summary
    (FETCH_SIZE and WRITE_SIZE, each scaled by what the counter reads for a plain
    1 GiB copy), or None when there is none for this workload or the kernel's
    sources changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "k_march_cells_c3_counters.txt")
    if config != "C3" or not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        line = line.strip()
        if line and not line.startswith("#") and "=" in line:
            k, v = line.split("=", 1)
            kv[k.strip()] = v.strip()
    h = hashlib.sha256()
    for f in kv.get("sources", "").split():
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    if h.hexdigest() != kv.get("sources_sha256"):
        return None
    fetch = float(kv["fetch_kib_per_dispatch"]) * (1048576.0 / float(kv["copy_fetch_kib_per_gib"]))
    write = float(kv["write_kib_per_dispatch"]) * (1048576.0 / float(kv["copy_write_kib_per_gib"]))
    hit = None
    if "tcc_hit_per_dispatch" in kv and "tcc_miss_per_dispatch" in kv:
        h, m = float(kv["tcc_hit_per_dispatch"]), float(kv["tcc_miss_per_dispatch"])
        hit = h / (h + m) if h + m > 0 else None
    return int((fetch + write) * 1024), hit


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", default="C3", choices=["C2", "C3"])
    ap.add_argument("--views", type=int, default=0, help="views per step (default: the config's)")
    ap.add_argument("--tf", default="ramp", choices=["ramp", "suppress"])
    ap.add_argument("--materialize", action="store_true")
    ap.add_argument("--macrocell", type=int, default=16,
                    help="macrocell edge for empty-space skipping (0: none; used by tables with zero opacity)")
    ap.add_argument("--tile", type=int, default=0)
    ap.add_argument("--twin", type=int, default=1,
                    help="1: keep a permuted copy of the cube for views along axis 1 (one more cube of HBM)")
    ap.add_argument("--oracle-seconds", type=float, default=15.0)
    ap.add_argument("--no-oracle", action="store_true")
    ap.add_argument("--per-view", action="store_true", help="print each view's march time to stderr")
    ap.add_argument("--no-extras", action="store_true", help="skip every leg besides the headline march")
    ap.add_argument("--legs", default="variants,tf_suppress,batched,fwd_bwd,c2",
                    help="comma-separated extra legs to run (variants = perspective, MIP, whole-ray termination)")
    ap.add_argument("--traffic-model", action="store_true",
                    help="only print the footprint-cell march's window-traffic model for the config's views "
                         "(host planning, no GPU)")
    ap.add_argument("--copy-probe", type=float, default=0.0,
                    help="only run a device-to-device copy of this many GiB (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: this build renders on a single MI355X "
              "(multi-GPU sort-last compositing is a design, not an implementation)", file=sys.stderr)
        sys.exit(2)

    if args.traffic_model:
        print(json.dumps(traffic_model(args.config, bool(args.twin))))
        return
    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.copy_probe > 0:
        nbytes = int(args.copy_probe * 2**30)
        x = torch.ones(nbytes // 4, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_read": nbytes, "copy_probe_bytes_written": nbytes, "launches": 3}))
        return
    cfg = synth.CONFIGS[args.config]
    n1, n2, n3 = cfg["dims"]
    W, H = cfg["image"]
    nviews = args.views or cfg["nviews"]
    t0 = time.time()
    log(f"generating {args.config} cube {n1}x{n2}x{n3} ({n1 * n2 * n3 * 4 / 2**30:.1f} GiB)")
    vol = synth.config_cube(args.config)
    log(f"generated in {time.time() - t0:.1f} s")

    ctx = vr.vr_create(0)
    t0 = time.time()
    h = vr.vr_volume_create(ctx, vol, (n1, n2, n3), on_device=False)
    vmin, vmax = vr.vr_volume_minmax(h)
    log(f"uploaded + min/max in {time.time() - t0:.1f} s: range [{vmin:.3f}, {vmax:.3f}]")
    t0 = time.time()
    vr.vr_volume_brick(h, vr.grid_spec(cfg["bricks"], materialize=args.materialize, macrocell=args.macrocell,
                                       twin=bool(args.twin)))
    bricks = vr.vr_volume_brick_info(h)
    log(f"bricked into {len(bricks)} bricks in {time.time() - t0:.1f} s")
    if args.tf == "ramp":
        tf = synth.tf_ramp(256)
    else:
        tf = synth.tf_noise_suppress(vmin, vmax, thresh=6.0)
    vr.vr_tf_set(ctx, tf)
    views_R = synth.random_views(nviews, cfg["view_seed"])
    views = [vr.make_view(R, W, H) for R in views_R]
    params = vr.make_params(step=0.5, tau=0.99, ess=1, tile=args.tile)
    nominal = sum(vr.vr_count_samples((n1, n2, n3), v, 0.5) for v in views)
    log(f"nominal samples per step: {nominal:.4g} ({nominal / nviews:.4g} per frame)")

    out = torch.empty((nviews, H, W, 4), device="cuda")
    stream = torch.cuda.current_stream()
    for _ in range(args.warmup):
        vr.vr_render(ctx, h, views, params, out, stream)
    torch.cuda.synchronize()

    # march launches: per-view algorithmic bytes (interior voxels of the bricks
    # rendered + brick-image writes), from the host plan (the same rectangles and
    # the same transparent-brick test as the renderer; no kernel runs for it)
    imgs_per_view = alg_bytes_per_view((n1, n2, n3), cfg["bricks"], bricks, views, tf, vmin, vmax)

    # one view per call, before the timed region: the spread of the march time
    # over view directions (the paper reports min / average / max over orientations)
    view_ms = []
    vr.vr_set_profiling(ctx, True)
    for i, v in enumerate(views):
        o1 = out[i:i + 1]
        vr.vr_render(ctx, h, [v], params, o1, stream)
        ms, cnt = vr.vr_stage_times(ctx)
        view_ms.append(ms[vr.VR_STAGE_MARCH])
        if args.per_view:
            d = views_R[i][2]
            log(f"view {i:2d} dir ({d[0]:+.3f},{d[1]:+.3f},{d[2]:+.3f}): march {ms[vr.VR_STAGE_MARCH]:.3f} ms")
    vr.vr_set_profiling(ctx, False)

    vr.vr_set_profiling(ctx, True)
    march_ms = []
    comp_ms = []
    setup_ms = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        vr.vr_render(ctx, h, views, params, out, stream)
        ms, cnt = vr.vr_stage_times(ctx)
        march_ms.append(ms[vr.VR_STAGE_MARCH] / max(1, cnt[vr.VR_STAGE_MARCH]))
        comp_ms.append(ms[vr.VR_STAGE_COMPOSITE] / max(1, cnt[vr.VR_STAGE_COMPOSITE]))
        setup_ms.append(ms[vr.VR_STAGE_SETUP] / nviews)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    vr.vr_set_profiling(ctx, False)
    ms_step = 1e3 * elapsed / args.steps
    gsps = nominal * args.steps / elapsed / 1e9
    avg_march = float(np.mean(march_ms))
    alg_bytes = float(np.mean([b + i for b, i, _ in imgs_per_view]))
    achieved = alg_bytes / (avg_march * 1e-3) / 1e9
    peak_meas = stream_peak(stream)
    traffic = counter_traffic(args.config)
    log(f"measured stream peak (device copy, reads + writes): {peak_meas:.0f} GB/s")
    log(f"{ms_step:.2f} ms/step, {ms_step / nviews:.3f} ms/frame, {gsps:.1f} Gsamples/s; "
        f"march {avg_march:.3f} ms/launch, composite {float(np.mean(comp_ms)):.3f} ms/launch")

    result = {
        "metric": METRIC,
        "value": round(gsps, 3),
        "unit": "Gsamples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"{args.config}: {n1}x{n2}x{n3} f32 cube ({n1 * n2 * n3 * 4 / 2**30:.1f} GiB), "
                        f"{cfg['bricks'][0]}^3 bricks, {W}x{H} frames, {nviews} views/step, step 0.5, "
                        f"tau 0.99 local ERT, TF {args.tf}" + (", materialised bricks" if args.materialize else "")
                        + (", permuted copy for views along axis 1" if args.twin else ""),
            "volume": [n1, n2, n3], "bricks": list(cfg["bricks"]), "image": [W, H], "views_per_step": nviews,
            "tf": args.tf, "tile": args.tile or 8, "macrocell": args.macrocell, "twin": bool(args.twin),
        },
        "ms_per_frame": round(ms_step / nviews, 4),
        "nominal_samples_per_frame": int(nominal // nviews),
        "march_ms_per_launch": round(avg_march, 4),
        "composite_ms_per_launch": round(float(np.mean(comp_ms)), 4),
        "setup_ms_per_frame": round(float(np.mean(setup_ms)), 4),
        "frame_time_decomposition": "ms_per_frame = setup (per-view tables to the device) + march + composite "
                                    "+ host gaps; the cube's upload, bricking and ranges are done once, "
                                    "before timing",
        "bricks_rendered_per_frame": float(np.mean([k for _, _, k in imgs_per_view])),
        "march_ms_per_view": {"min": round(float(np.min(view_ms)), 4), "median": round(float(np.median(view_ms)), 4),
                              "mean": round(float(np.mean(view_ms)), 4), "max": round(float(np.max(view_ms)), 4),
                              "views": len(view_ms), "how": "one view per call, between the warm-up and the timed steps"},
        "roofline": {
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic[0] if traffic else None,
            "traffic_source": "rocprofv3 FETCH_SIZE + WRITE_SIZE per dispatch (L2-miss traffic, scaled by a "
                              "plain copy), read from profiles/k_march_cells_c3_counters.txt when the kernel and "
                              "planning sources hash to the values recorded there, else null",
            "l2_hit_rate": round(traffic[1], 4) if traffic and traffic[1] is not None else None,
            "kernel": "k_march_cells",
            "alg_bytes_per_launch": int(alg_bytes),
            "measured_stream_peak": round(peak_meas, 1),
            "frac_of_measured_peak": round(achieved / peak_meas, 4),
            "valu_frac": round(LANE_OPS_PER_SAMPLE * (nominal / nviews) / (avg_march * 1e-3) / VALU_PEAK_LANE_OPS, 4),
        },
    }

    legs = set() if args.no_extras else set(args.legs.split(","))
    if "variants" in legs:
        result.update(bench_variants(ctx, h, (n1, n2, n3), views_R, W, H, stream, (cfg["bricks"], bricks, tf, vmin, vmax)))
    if "tf_suppress" in legs:
        result["tf_suppress"] = bench_tf_suppress(ctx, h, (n1, n2, n3), views_R, W, H, vmin, vmax, stream)
    if "batched" in legs:
        result["batched"] = bench_batched(ctx, stream)
    if "fwd_bwd" in legs:
        result["fwd_bwd"] = bench_fwd_bwd(ctx, stream)
    if "c2" in legs and args.config == "C3":
        result["c2"] = bench_c2(ctx, stream)

    if not args.no_oracle:
        import oracle
        oracle.lib()
        got = out.cpu().numpy()
        rng = np.random.Generator(np.random.PCG64(7))
        cores = threads_used()
        # bounded sample: strided rays (every 4th row and column) of successive views,
        # until the time budget is spent
        stride = 4
        done_rays = 0
        done_samples = 0
        done_eval = 0
        spent = 0.0
        worst = 0.0
        nv_done = 0
        for vi in range(nviews):
            yy, xx = np.meshgrid(np.arange(int(rng.integers(stride)), H, stride),
                                 np.arange(int(rng.integers(stride)), W, stride), indexing="ij")
            vv = np.full(yy.size, vi, np.int32)
            t1 = time.perf_counter()
            ref = oracle.render_rays(vol, tf, [views_R[vi]], W, H, np.zeros(yy.size, np.int32), xx.ravel(),
                                     yy.ravel(), vmin, vmax, tau=0.99, bricks={"grid": cfg["bricks"]},
                                     nthreads=cores)
            spent += time.perf_counter() - t1
            nv_done += 1
            done_rays += yy.size
            done_samples += int(ref["nsamples"].sum())
            done_eval += int(ref["neval"].sum())
            g = got[vv, yy.ravel(), xx.ravel()].astype(np.float64)
            ok = (ref["flags"] & oracle.FLAG_GEOM) == 0
            e = oracle.match_error(g, ref)[ok]
            worst = max(worst, float(e.max()) if e.size else 0.0)
            if spent >= args.oracle_seconds:
                break
        result["cpu_baseline"] = {
            "value": round(done_samples / spent / 1e9, 5),
            "unit": "Gsamples/s",
            "cores": cores,
            "kind": "oracle",
            "sample": f"{done_rays} rays (every {stride}th row and column of {nv_done} of the {nviews} views), "
                      f"{done_samples} nominal samples, FP64, {spent:.1f} s",
        }
        result["parity_max_err_on_sample"] = float(f"{max(worst, 0.0):.3g}")
        frac_eval = done_eval / max(1, done_samples)
        result["effective_samples_per_frame"] = int(frac_eval * (nominal // nviews))
        result["effective_samples_how"] = (f"nominal x {frac_eval:.4f}, the fraction of lattice samples evaluated "
                                           "(each brick's samples up to its own early termination) on the oracle's "
                                           "ray sample")
        log(f"oracle: {done_samples / spent / 1e6:.1f} Msamples/s on {cores} threads; parity {worst:.3g}")

    vr.vr_volume_destroy(h)
    vr.vr_destroy(ctx)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
