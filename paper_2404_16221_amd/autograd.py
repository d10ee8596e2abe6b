"""torch.autograd.Functions over the C ABI: partitioned rendering and feature
channels, forward and backward.

XLRender -- forward: per-segment composite (xl_render_segments_fwd), then the
merge in ray order (xl_merge_fwd).  Backward: merge backward (xl_merge_bwd)
into each segment's tuple gradient, then the per-segment backward
(xl_render_segments_bwd) into sigma and rgb.

XLFeatures -- the same for F feature channels rendered with the
volume-rendering weights (App. B.2): xl_render_features_fwd,
xl_merge_features_fwd, and their backwards into sigma and the features.  When
both are used on the same sigma, autograd adds the two density gradients.

Gradients flow to sigma, rgb and the features only (interval ends are data,
not parameters).
"""
from __future__ import annotations

import torch

from . import _lib


class XLRender(torch.autograd.Function):
    @staticmethod
    def forward(ctx, sigma, rgb, t_start, t_end, seg_offsets, ray_offsets, seg_ids, fp64=False,
                region_offsets=None):
        seg_out, ws = _lib.xl_render_segments_fwd(sigma, rgb, t_start, t_end, seg_offsets)
        ray_out = _lib.xl_merge_fwd(seg_out, ray_offsets, seg_ids, fp64=fp64,
                                    region_offsets=region_offsets)
        ctx.save_for_backward(sigma, rgb, t_start, t_end, seg_offsets, ray_offsets, seg_ids,
                              seg_out, ws)
        ctx.fp64 = fp64
        ctx.region_offsets = region_offsets
        return ray_out

    @staticmethod
    def backward(ctx, grad_ray):
        sigma, rgb, t_start, t_end, seg_offsets, ray_offsets, seg_ids, seg_out, ws = ctx.saved_tensors
        grad_ray = grad_ray.to(torch.float32).contiguous()
        grad_seg = _lib.xl_merge_bwd(seg_out, ray_offsets, seg_ids, grad_ray, fp64=ctx.fp64,
                                     region_offsets=ctx.region_offsets)
        gs, gc = _lib.xl_render_segments_bwd(sigma, rgb, t_start, t_end, seg_offsets, ws, grad_seg)
        return gs, gc, None, None, None, None, None, None, None


def render(sigma, rgb, t_start, t_end, seg_offsets, ray_offsets, seg_ids, fp64=False,
           region_offsets=None):
    """ray tuple [7, n_rays] = (T, r, g, b, A, D, L), differentiable in sigma and rgb.
    region_offsets [K + 1] (optional): the segments' region boundaries, which
    let the merge stage each workgroup's tuples through LDS."""
    return XLRender.apply(sigma, rgb, t_start, t_end, seg_offsets, ray_offsets, seg_ids, fp64,
                          region_offsets)


class XLFeatures(torch.autograd.Function):
    @staticmethod
    def forward(ctx, sigma, feat, t_start, t_end, seg_offsets, ray_offsets, seg_ids):
        phi, tau = _lib.xl_render_features_fwd(sigma, feat, t_start, t_end, seg_offsets)
        out = _lib.xl_merge_features_fwd(tau, phi, ray_offsets, seg_ids)
        ctx.save_for_backward(sigma, feat, t_start, t_end, seg_offsets, ray_offsets, seg_ids, phi, tau)
        return out

    @staticmethod
    def backward(ctx, grad_out):
        sigma, feat, t_start, t_end, seg_offsets, ray_offsets, seg_ids, phi, tau = ctx.saved_tensors
        grad_out = grad_out.to(torch.float32).contiguous()
        gphi, gtau = _lib.xl_merge_features_bwd(tau, phi, ray_offsets, seg_ids, grad_out)
        gs, gf = _lib.xl_render_features_bwd(sigma, feat, t_start, t_end, seg_offsets, phi, gphi, gtau)
        return gs, gf, None, None, None, None, None


def render_features(sigma, feat, t_start, t_end, seg_offsets, ray_offsets, seg_ids):
    """Per-ray features [F, n_rays] (F = feat.shape[1] in {4, 8, 16, 32}),
    differentiable in sigma and feat."""
    return XLFeatures.apply(sigma, feat, t_start, t_end, seg_offsets, ray_offsets, seg_ids)
