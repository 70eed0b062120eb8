"""The allocation-free batched entry point (vr_render_batch_noalloc) against
vr_render_batch, through the C ABI: two calls in a row on one context, the
second with fewer requests, each bit-identical to the graph-replayed batch;
requests beyond the fixed scratch's limit are refused before any GPU work."""
import numpy as np
import pytest

import paper_1008_0135_amd as vr
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu] {msg}", flush=True)


def _setup(ctx, descs):
    vols, reqs, outs, keep = [], [], [], []
    for d in descs:
        n1, n2, n3 = d["dims"]
        a = synth.cube(n1, n2, n3, seed=d["seed"], n_sources=d["n_sources"], sigma_range=(1.5, 3.0))
        vols.append(vr.vr_volume_create(ctx, a, (n1, n2, n3)))
        W, H = d["image"]
        t = torch.from_numpy(d["tf"]).cuda()
        o = torch.full((H, W, 4), -1.0, device="cuda")
        keep.append(t)
        outs.append(o)
        reqs.append(vr.make_request(vols[-1], d["view"], W, H, t, 0.0, 0.0, o))
    return vols, reqs, outs, keep


def test_noalloc_batch_matches_batch():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ctx = vr.vr_create(0)
    try:
        params = vr.make_params(tau=0.99)
        descs = synth.batch_requests(seed=91, nreq=12, dim_range=(20, 90), img_range=(9, 130))
        vols, reqs, outs, keep = _setup(ctx, descs)
        for call, m in enumerate((12, 5)):
            _say(f"allocation-free batch, call {call + 1}: {m} requests")
            for o in outs:
                o.fill_(-1.0)
            vr.vr_render_batch_noalloc(ctx, reqs[:m], params)
            torch.cuda.synchronize()
            got = [o.cpu().numpy().copy() for o in outs[:m]]
            for o in outs:
                o.fill_(-2.0)
            cache = vr.vr_render_batch(ctx, reqs[:m], params, None)
            torch.cuda.synchronize()
            for i in range(m):
                want = outs[i].cpu().numpy()
                assert (want >= 0).all(), (call, i)
                assert np.array_equal(got[i], want), (call, i)
            vr.vr_batch_destroy(cache)
        # beyond the fixed scratch: refused on the host
        big = [reqs[0]] * 513
        with pytest.raises(RuntimeError, match="513 requests exceed"):
            vr.vr_render_batch_noalloc(ctx, big, params)
        for v in vols:
            vr.vr_volume_destroy(v)
        del keep
    finally:
        vr.vr_destroy(ctx)
