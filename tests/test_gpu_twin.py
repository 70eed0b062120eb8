"""GPU checks of the permuted copy used for views along axis 1 (through the C ABI).

* views looking mostly along axis 1 (orthographic and perspective; grid,
  longest-axis and materialised bricks; emission-absorption with per-brick or
  whole-ray termination, macrocell skipping, and MIP) match the FP64 oracle
  when rendered from the copy;
* other views give the same bits with and without the copy;
* bricking again without the copy drops it.
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


def _render(ctx, h, views, W, H, params, eye=0.0):
    out = torch.full((len(views), H, W, 4), -7.0, device="cuda")
    vr.vr_render(ctx, h, [vr.make_view(R, W, H, eye_dist=eye) for R in views], params, out)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def _axis1_views(seed, n):
    """Rotations whose viewing direction is closest to axis 1 (either sign)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    while len(out) < n:
        R = synth.random_rotation(rng)
        if abs(R[2][0]) > max(abs(R[2][1]), abs(R[2][2])):
            out.append(R)
    return out


DIMS = (90, 84, 100)
LAYOUTS = {"grid": ((40, 36, 48), None), "kd": (None, 7), "mat": ((45, 42, 50), None)}


def _spec(name, twin, macrocell=0):
    size, kd = LAYOUTS[name]
    if kd:
        return vr.kd_spec(kd, twin=twin, macrocell=macrocell)
    return vr.grid_spec(size, materialize=name == "mat", twin=twin, macrocell=macrocell)


def _oracle_bricks(name):
    size, kd = LAYOUTS[name]
    return oracle.kd_boxes(DIMS, kd) if kd else {"grid": size}


@pytest.mark.parametrize("layout,eye,mode,scope", [("grid", 0.0, 0, 0), ("kd", 0.0, 0, 0), ("mat", 0.0, 0, 0),
                                                   ("grid", 110.0, 0, 0), ("kd", 0.0, 1, 0), ("grid", 0.0, 0, 1),
                                                   ("kd", 130.0, 0, 1)])
def test_axis1_views_from_copy_match_oracle(ctx, layout, eye, mode, scope):
    _say(f"permuted copy: {layout} eye {eye} mode {mode} scope {scope}")
    vol = synth.cube(*DIMS, seed=131, n_sources=8, sigma_range=(2.0, 4.0))
    h = vr.vr_volume_create(ctx, vol, DIMS)
    vr.vr_volume_brick(h, _spec(layout, True, macrocell=8))
    mn, mx = float(vol.min()), float(vol.max())
    tf = synth.tf_colour(256)
    tf[:, 3] = np.minimum(1.0, tf[:, 3] * 8)
    vr.vr_tf_set(ctx, tf, mn, mx)
    views = _axis1_views(132, 3)
    p = vr.make_params(tau=0.99, mode=mode, ert_scope=scope)
    img = _render(ctx, h, views, 112, 96, p, eye)
    ref = oracle.render(vol, tf, views, 112, 96, mn, mx, tau=0.99, mode=mode, eye_dist=eye,
                        bricks=None if scope else _oracle_bricks(layout))
    _say(f"  {parity(img, ref, label=f'copy {layout}')}")
    vr.vr_volume_destroy(h)


def test_copy_changes_nothing_elsewhere_and_is_dropped(ctx):
    _say("permuted copy: other views bit-identical; bricking without it drops it")
    dims = (120, 100, 140)
    vol = synth.cube(*dims, seed=133, n_sources=10, sigma_range=(2.0, 4.0))
    mn, mx = float(vol.min()), float(vol.max())
    vr.vr_tf_set(ctx, synth.tf_noise_suppress(mn, mx, thresh=4.0, amax=0.3), mn, mx)
    rng = np.random.Generator(np.random.PCG64(134))
    views = []
    while len(views) < 4:
        R = synth.random_rotation(rng)
        if abs(R[2][0]) < max(abs(R[2][1]), abs(R[2][2])):
            views.append(R)
    spec_args = dict(size=(48, 40, 56), macrocell=8)
    plain = vr.vr_volume_create(ctx, vol, dims)
    vr.vr_volume_brick(plain, vr.grid_spec(**spec_args))
    twin = vr.vr_volume_create(ctx, vol, dims)
    vr.vr_volume_brick(twin, vr.grid_spec(**spec_args, twin=True))
    for eye in (0.0, 150.0):
        a = _render(ctx, plain, views, 128, 112, vr.make_params(), eye)
        b = _render(ctx, twin, views, 128, 112, vr.make_params(), eye)
        assert np.array_equal(a, b)
    # mixed calls: views along axis 1 and others in one call, in any order
    mixed = [views[0]] + _axis1_views(135, 2) + [views[1]]
    m = _render(ctx, twin, mixed, 96, 80, vr.make_params())
    for i, R in enumerate(mixed):
        single = _render(ctx, twin, [R], 96, 80, vr.make_params())
        assert np.array_equal(m[i], single[0])
    vr.vr_volume_brick(twin, vr.grid_spec(**spec_args))  # no copy any more
    ax = _axis1_views(136, 2)
    assert np.array_equal(_render(ctx, twin, ax, 96, 80, vr.make_params()),
                          _render(ctx, plain, ax, 96, 80, vr.make_params()))
    vr.vr_volume_destroy(plain)
    vr.vr_volume_destroy(twin)
