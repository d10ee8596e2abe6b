"""torch.autograd.Function over the C ABI: partitioned rendering, forward and backward.

Forward: per-segment composite (xl_render_segments_fwd), then the merge in ray
order (xl_merge_fwd).  Backward: merge backward (xl_merge_bwd) into each
segment's tuple gradient, then the per-segment backward
(xl_render_segments_bwd) into sigma and rgb.  Gradients flow to sigma and rgb
only (interval ends are data, not parameters).
"""
from __future__ import annotations

import torch

from . import _lib


class XLRender(torch.autograd.Function):
    @staticmethod
    def forward(ctx, sigma, rgb, t_start, t_end, seg_offsets, ray_offsets, seg_ids, fp64=False):
        seg_out, ws = _lib.xl_render_segments_fwd(sigma, rgb, t_start, t_end, seg_offsets)
        ray_out = _lib.xl_merge_fwd(seg_out, ray_offsets, seg_ids, fp64=fp64)
        ctx.save_for_backward(sigma, rgb, t_start, t_end, seg_offsets, ray_offsets, seg_ids,
                              seg_out, ws)
        ctx.fp64 = fp64
        return ray_out

    @staticmethod
    def backward(ctx, grad_ray):
        sigma, rgb, t_start, t_end, seg_offsets, ray_offsets, seg_ids, seg_out, ws = ctx.saved_tensors
        grad_ray = grad_ray.to(torch.float32).contiguous()
        grad_seg = _lib.xl_merge_bwd(seg_out, ray_offsets, seg_ids, grad_ray, fp64=ctx.fp64)
        gs, gc = _lib.xl_render_segments_bwd(sigma, rgb, t_start, t_end, seg_offsets, ws, grad_seg)
        return gs, gc, None, None, None, None, None, None


def render(sigma, rgb, t_start, t_end, seg_offsets, ray_offsets, seg_ids, fp64=False):
    """ray tuple [7, n_rays] = (T, r, g, b, A, D, L), differentiable in sigma and rgb."""
    return XLRender.apply(sigma, rgb, t_start, t_end, seg_offsets, ray_offsets, seg_ids, fp64)
