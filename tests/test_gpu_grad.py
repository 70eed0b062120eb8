"""GPU parity of the differentiable path (adjoint march) through the C ABI.

* the checkpointing forward gives the same image bits as the plain forward;
* table and voxel gradients vs the FP64 oracle's exact gradient (relative
  error <= 1e-3 with the scale floor 1e-3 * max|g|), for several checkpoint
  intervals, with and without early termination;
* table gradients vs central finite differences of the FP64 forward (eps = 1e-3,
  the configuration's table), and vs Richardson-extrapolated differences for a
  high-opacity table whose plain differences are not accurate to 1e-3;
* the torch.autograd.Function on an L2 loss against a perturbed-table target;
* the 256x256x512 / 512^2 case on 2 of its 8 views.
"""
import numpy as np
import pytest

import oracle
import paper_1008_0135_amd as vr
import synth

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


def _rel(g, ref):
    scale = max(1e-3 * float(np.abs(ref).max()), 1e-30)
    return np.abs(g - ref) / np.maximum(np.abs(ref), scale)


def _case(seed=41, dims=(48, 40, 56), M=64, amul=3.0):
    vol = synth.cube(*dims, seed=seed, n_sources=4, sigma_range=(2.0, 4.0))
    tf = synth.tf_colour(M)
    tf[:, 3] = np.minimum(1.0, tf[:, 3] * amul)
    vmin, vmax = float(vol.min()) - 0.5, float(vol.max()) + 0.5
    return vol, tf, vmin, vmax


def _gpu_grad(ctx, vol, tf, views, W, H, vmin, vmax, gout, tau=2.0, K=32):
    n3, n2, n1 = vol.shape
    dvol = torch.from_numpy(vol).cuda()
    h = vr.vr_volume_wrap(ctx, dvol, (n1, n2, n3))
    vr.vr_tf_set(ctx, tf, vmin, vmax)
    out = torch.empty((len(views), H, W, 4), device="cuda")
    p = vr.make_params(tau=tau, ckpt_K=K, ess=0)
    vv = [vr.make_view(R, W, H) for R in views]
    st = vr.vr_render(ctx, h, vv, p, out, save=True)
    plain = torch.empty_like(out)
    vr.vr_render(ctx, h, vv, p, plain)
    g = torch.from_numpy(np.ascontiguousarray(gout, np.float32)).cuda()
    gtf = torch.empty((tf.shape[0], 4), device="cuda")
    gvol = torch.empty_like(dvol)
    vr.vr_render_backward(ctx, h, st, g, gtf, gvol)
    torch.cuda.synchronize()
    res = (out.cpu().numpy(), plain.cpu().numpy(), gtf.cpu().numpy().astype(np.float64),
           gvol.cpu().numpy().astype(np.float64))
    vr.vr_state_destroy(st)
    vr.vr_volume_destroy(h)
    return res


def _oracle_grad(vol, tf, views, W, H, vmin, vmax, gout, tau=2.0):
    gtf = np.zeros((tf.shape[0], 4))
    gvol = np.zeros(vol.shape)
    imgs = []
    for j, R in enumerate(views):
        a, b, img = oracle.render_grad(vol, tf, R, W, H, gout[j], vmin, vmax, tau=tau)
        gtf += a
        gvol += b
        imgs.append(img)
    return gtf, gvol, np.stack(imgs)


@pytest.mark.parametrize("K", [32, 7, 1, 64])
def test_gradients_match_oracle(ctx, K):
    _say(f"adjoint vs FP64 oracle, K = {K}")
    vol, tf, vmin, vmax = _case()
    views = synth.random_views(2, 42)
    W = H = 64
    rng = np.random.Generator(np.random.PCG64(43))
    gout = rng.normal(0, 1, (2, H, W, 4))
    img, plain, gtf, gvol = _gpu_grad(ctx, vol, tf, views, W, H, vmin, vmax, gout, K=K)
    assert np.array_equal(img, plain)
    otf, ovol, oimg = _oracle_grad(vol, tf, views, W, H, vmin, vmax, gout)
    assert np.abs(img - oimg).max() <= 2e-5
    r_tf = _rel(gtf, otf)
    r_vol = _rel(gvol, ovol)
    _say(f"max rel err: tf {r_tf.max():.3g}, voxels {r_vol.max():.3g}")
    assert r_tf.max() <= 1e-3
    assert r_vol.max() <= 1e-3


def test_gradients_with_early_termination(ctx):
    _say("adjoint with ERT (frozen termination index)")
    vol, tf, vmin, vmax = _case(seed=44, amul=20.0)
    views = synth.random_views(2, 45)
    W = H = 64
    rng = np.random.Generator(np.random.PCG64(46))
    gout = rng.normal(0, 1, (2, H, W, 4))
    # rays whose opacity lands within rounding of tau may stop one sample apart on
    # the two sides: give them no upstream gradient so both sides exclude them
    ref = oracle.render(vol, tf, views, W, H, vmin, vmax, tau=0.95)
    tie = (ref["flags"] & oracle.FLAG_ERT) != 0
    gout[tie] = 0.0
    img, plain, gtf, gvol = _gpu_grad(ctx, vol, tf, views, W, H, vmin, vmax, gout, tau=0.95)
    otf, ovol, oimg = _oracle_grad(vol, tf, views, W, H, vmin, vmax, gout, tau=0.95)
    assert np.abs(img - oimg)[~tie].max() <= 2e-5
    assert (1.0 - img[..., 3] <= 0.05 + 1e-6).mean() > 0.2  # termination fired on many rays
    assert _rel(gtf, otf).max() <= 1e-3
    assert _rel(gvol, ovol).max() <= 1e-3


def _fd_case(tf):
    vol = synth.cube(24, 20, 28, seed=47, n_sources=4, sigma_range=(2.0, 4.0))
    vmin, vmax = float(vol.min()) - 0.5, float(vol.max()) + 0.5
    views = synth.random_views(2, 48)
    W = H = 24
    target = np.stack([oracle.render(vol, synth.tf_perturbed(tf, 49), [R], W, H, vmin, vmax, tau=2.0)["image"][0]
                       for R in views])
    base = np.stack([oracle.render(vol, tf, [R], W, H, vmin, vmax, tau=2.0)["image"][0] for R in views])

    def loss(t):
        img = np.stack([oracle.render(vol, t, [R], W, H, vmin, vmax, tau=2.0)["image"][0] for R in views])
        return 0.5 * float(((img - target) ** 2).sum())

    def fd(eps):
        out = np.zeros(tf.shape)
        for i in range(tf.shape[0]):
            for c in range(4):
                tp = tf.astype(np.float64).copy()
                tm = tp.copy()
                tp[i, c] += eps
                tm[i, c] -= eps
                tp32, tm32 = tp.astype(np.float32), tm.astype(np.float32)
                out[i, c] = (loss(tp32) - loss(tm32)) / (float(tp32[i, c]) - float(tm32[i, c]))
        return out

    return vol, views, W, H, vmin, vmax, base - target, fd


def test_tf_gradient_vs_central_fd(ctx):
    """Configuration protocol: central differences of the FP64 forward, eps = 1e-3, every entry
    of the configuration's table (colour ramp, alpha = 0.02 t, 256 entries)."""
    _say("adjoint vs central finite differences (eps = 1e-3)")
    tf = synth.tf_colour(256)
    vol, views, W, H, vmin, vmax, gout, fd = _fd_case(tf)
    _, _, gtf, _ = _gpu_grad(ctx, vol, tf, views, W, H, vmin, vmax, gout)
    r = _rel(gtf, fd(1e-3))
    _say(f"max rel err vs FD: {r.max():.3g}")
    assert r.max() <= 1e-3


def test_tf_gradient_vs_extrapolated_fd(ctx):
    """High-opacity 16-entry table, where plain central FD at eps = 1e-3 carries ~3e-3 of its own
    O(eps^2) truncation error: compare with the Richardson extrapolation of eps and eps/2."""
    _say("adjoint vs Richardson-extrapolated finite differences")
    tf = synth.tf_colour(16)
    tf[:, 3] = np.minimum(1.0, tf[:, 3] * 2)
    vol, views, W, H, vmin, vmax, gout, fd = _fd_case(tf)
    _, _, gtf, _ = _gpu_grad(ctx, vol, tf, views, W, H, vmin, vmax, gout)
    rich = (4.0 * fd(5e-4) - fd(1e-3)) / 3.0
    r = _rel(gtf, rich)
    _say(f"max rel err vs extrapolated FD: {r.max():.3g}")
    assert r.max() <= 1e-3


def test_autograd_function_l2_loss(ctx):
    _say("torch.autograd.Function: L2 loss vs perturbed-table target")
    from paper_1008_0135_amd.autograd import render
    vol, tf, vmin, vmax = _case(seed=50)
    views = synth.random_views(2, 51)
    W = H = 48
    vv = [vr.make_view(R, W, H) for R in views]
    target_tf = synth.tf_perturbed(tf, 52)
    target = np.stack([oracle.render(vol, target_tf, [R], W, H, vmin, vmax, tau=2.0)["image"][0] for R in views])
    v = torch.from_numpy(vol).cuda().requires_grad_(True)
    t = torch.from_numpy(tf).cuda().requires_grad_(True)
    img = render(v, t, vv, ctx, vmin, vmax, ckpt_K=16)
    loss = 0.5 * ((img - torch.from_numpy(target).float().cuda()) ** 2).sum()
    loss.backward()
    gout = img.detach().cpu().numpy().astype(np.float64) - target
    otf, ovol, _ = _oracle_grad(vol, tf, views, W, H, vmin, vmax, gout)
    assert _rel(t.grad.cpu().numpy().astype(np.float64), otf).max() <= 1e-3
    assert _rel(v.grad.cpu().numpy().astype(np.float64), ovol).max() <= 1e-3


def test_c5_full_size_two_views(ctx):
    """256x256x512, 512^2: forward + adjoint on the GPU, FP64 gradient on 2 views."""
    _say("C5: 256x256x512 volume, 2 views at 512^2")
    c = synth.CONFIGS["C5"]
    vol = synth.config_cube("C5")
    tf = synth.tf_colour(256)
    vmin, vmax = float(vol.min()) - 0.5, float(vol.max()) + 0.5
    views = synth.random_views(c["nviews"], c["view_seed"])[:2]
    W, H = c["image"]
    target = np.stack([oracle.render(vol, synth.tf_perturbed(tf, c["tf_seed"]), [R], W, H, vmin, vmax,
                                     tau=2.0)["image"][0] for R in views])
    base = np.stack([oracle.render(vol, tf, [R], W, H, vmin, vmax, tau=2.0)["image"][0] for R in views])
    gout = base - target
    img, plain, gtf, gvol = _gpu_grad(ctx, vol, tf, views, W, H, vmin, vmax, gout)
    assert np.abs(img - base).max() <= 2e-5
    otf, ovol, _ = _oracle_grad(vol, tf, views, W, H, vmin, vmax, gout)
    r_tf, r_vol = _rel(gtf, otf), _rel(gvol, ovol)
    _say(f"C5 max rel err: tf {r_tf.max():.3g}, voxels {r_vol.max():.3g}")
    assert r_tf.max() <= 1e-3
    assert r_vol.max() <= 1e-3


def test_checkpoint_interval_follows_ckpt_K(ctx):
    """The planned checkpoint group follows ckpt_K: L = round(K step |d_b|) cell layers,
    capped at 3, so the interval is min(K, about 3 / (step |d_b|)) samples; gradients
    agree across intervals (the exact derivative does not depend on where the
    recomputation restarts)."""
    vol, tf, vmin, vmax = _case(seed=51)
    n3, n2, n1 = vol.shape
    dvol = torch.from_numpy(vol).cuda()
    h = vr.vr_volume_wrap(ctx, dvol, (n1, n2, n3))
    vr.vr_tf_set(ctx, tf, vmin, vmax)
    R = synth.random_views(1, 52)[0]
    W = H = 40
    view = vr.make_view(R, W, H)
    out = torch.empty((1, H, W, 4), device="cuda")
    g = torch.from_numpy(np.random.Generator(np.random.PCG64(53)).normal(0, 1, (1, H, W, 4)).astype(np.float32)).cuda()
    grads = {}
    for K in (2, 4, 8, 32, 64):
        st = vr.vr_render(ctx, h, [view], vr.make_params(tau=2.0, ckpt_K=K, ess=0), out, save=True)
        ring, L, spg = vr.vr_state_info(st, 0)
        assert ring
        d = np.abs(np.asarray(R, np.float64)[2])
        db = L / (0.5 * spg)  # |d_b| of the slab axis the plan took: axis 2 or 3
        assert min(abs(db - d[1]), abs(db - d[2])) <= 1e-9, (db, d)
        want = max(1, min(3, int(np.floor(K * 0.5 * db + 0.5))))
        assert L == want, (K, L, want)
        assert spg <= K + 1.0 / db + 1e-9, (K, L, spg)
        _say(f"ckpt_K {K}: {L} cell layers per group, {spg:.2f} samples per checkpoint")
        gtf = torch.empty((tf.shape[0], 4), device="cuda")
        gvol = torch.empty_like(dvol)
        vr.vr_render_backward(ctx, h, st, g, gtf, gvol)
        torch.cuda.synchronize()
        grads[K] = (gtf.cpu().numpy().astype(np.float64), gvol.cpu().numpy().astype(np.float64))
        vr.vr_state_destroy(st)
    for K in (2, 4, 8, 64):
        assert _rel(grads[K][0], grads[32][0]).max() <= 1e-4
        assert _rel(grads[K][1], grads[32][1]).max() <= 1e-4
    vr.vr_volume_destroy(h)


def _ctx_with_env(env):
    import os
    old = {k: os.environ.get(k) for k in env}
    os.environ.update(env)
    try:
        return vr.vr_create(0)
    finally:
        for k, v in old.items():
            if v is None:
                del os.environ[k]
            else:
                os.environ[k] = v


def test_adjoint_schedules_agree():
    """The differentiable pair's schedules (views side by side or one after
    another; tile groups in XCD bands of equal estimated work or equal counts)
    march the same tiles with the same arithmetic: the checkpointing forward's
    images are bit-identical and the gradients differ only by the order of
    their atomic and partial sums."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = synth.CONFIGS["C5"]
    vol = synth.config_cube("C5")
    tf = synth.tf_colour(256)
    vmin, vmax = float(vol.min()) - 0.5, float(vol.max()) + 0.5
    views = synth.random_views(c["nviews"], c["view_seed"])[:5]
    W, H = c["image"]
    gout = np.random.Generator(np.random.PCG64(71)).normal(0, 1, (len(views), H, W, 4)).astype(np.float32)
    res = {}
    for name, env in (("default", {}), ("in turn", {"VR_BWD_SIDE": "0"}), ("equal counts", {"VR_BWD_BANDS": "0"}),
                      ("both off", {"VR_BWD_SIDE": "0", "VR_BWD_BANDS": "0"})):
        _say(f"C5 volume, {len(views)} views at 512^2, schedule: {name}")
        cx = _ctx_with_env(env)
        try:
            res[name] = _gpu_grad(cx, vol, tf, views, W, H, vmin, vmax, gout)
        finally:
            vr.vr_destroy(cx)
    img0, plain0, gtf0, gvol0 = res["default"]
    for name, (img, plain, gtf, gvol) in res.items():
        assert np.array_equal(img, img0), name
        assert np.array_equal(plain, plain0), name
        r_tf, r_vol = _rel(gtf, gtf0), _rel(gvol, gvol0)
        _say(f"{name}: max rel difference tf {r_tf.max():.3g}, voxels {r_vol.max():.3g}")
        assert r_tf.max() <= 1e-5 and r_vol.max() <= 3e-4, name
