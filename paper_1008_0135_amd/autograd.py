"""torch.autograd.Function over libvr's differentiable render.

``render(volume, tf, views, ...)`` returns the [nviews][H][W][4] image and
differentiates it with respect to the voxel values and the transfer-function
table through the adjoint march of the library (transmittance checkpoints
every ``ckpt_K`` samples, segments replayed forward then walked backward).
The normalisation window [vmin, vmax] is a constant of the render.  Views
and parameters are not differentiable.  All arithmetic runs on the GPU in
the library; this module only passes tensors' device pointers and streams.
"""
from __future__ import annotations

import torch

import paper_1008_0135_amd as vr


class _Handles:
    """Library objects of one forward; released when backward ran or on collection."""

    def __init__(self, hctx, vol, state):
        self.hctx, self.vol, self.state = hctx, vol, state

    def release(self):
        if self.state:
            vr.vr_state_destroy(self.state)
            self.state = None
        if self.vol:
            vr.vr_volume_destroy(self.vol)
            self.vol = None

    def __del__(self):
        try:
            self.release()
        except Exception:
            pass


class VolumeRender(torch.autograd.Function):
    @staticmethod
    def forward(ctx, volume, tf, hctx, views, params, vmin, vmax):
        if not volume.is_cuda or volume.dtype != torch.float32 or volume.dim() != 3:
            raise ValueError("volume must be a float32 CUDA tensor [n3][n2][n1]")
        if not tf.is_cuda or tf.dtype != torch.float32 or tf.dim() != 2 or tf.shape[1] != 4:
            raise ValueError("tf must be a float32 CUDA tensor [M][4]")
        volume = volume.contiguous()
        tf = tf.contiguous()
        n3, n2, n1 = volume.shape
        stream = torch.cuda.current_stream()
        vol_h = vr.vr_volume_wrap(hctx, volume, (n1, n2, n3), stream)
        vr.vr_tf_set(hctx, tf.detach(), vmin, vmax, stream)
        W, H = views[0].W, views[0].H
        out = torch.empty((len(views), H, W, 4), device=volume.device, dtype=torch.float32)
        state = vr.vr_render(hctx, vol_h, views, params, out, stream, save=True)
        ctx.handles = _Handles(hctx, vol_h, state)
        ctx.save_for_backward(volume, tf)
        return out

    @staticmethod
    def backward(ctx, grad_out):
        volume, tf = ctx.saved_tensors
        h = ctx.handles
        stream = torch.cuda.current_stream()
        grad_out = grad_out.contiguous().float()
        gtf = torch.empty_like(tf)
        gvol = torch.empty_like(volume) if ctx.needs_input_grad[0] else None
        vr.vr_render_backward(h.hctx, h.vol, h.state, grad_out, gtf, gvol, accumulate=False, stream=stream)
        torch.cuda.current_stream().synchronize()
        h.release()
        return gvol, (gtf if ctx.needs_input_grad[1] else None), None, None, None, None, None


def render(volume, tf, views, hctx, vmin, vmax, step=0.5, tau=2.0, ckpt_K=32):
    """Differentiable render.  views: list of vr.vr_view (shared W, H).  tau >= 1 disables ERT."""
    params = vr.make_params(step=step, tau=tau, ess=0, ckpt_K=ckpt_K)
    return VolumeRender.apply(volume, tf, hctx, views, params, float(vmin), float(vmax))
