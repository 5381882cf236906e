"""PyTorch autograd wrapper around libgbr: images = BlendRender.apply(bases,
weights, cams, ctx).

Forward: blend (Eq. 1) of every frame's Gaussians, then the batched render
(Sec. 3.2).  Backward: the library's exact adjoint back to the bases and the
weights.  The library does all the work; this module only marshals tensors.

A context keeps the state of its last render for the backward (including a
pointer to the blended Gaussians, which the autograd context keeps alive), so
one forward may be in flight per context: call backward before the next
forward on the same context.  The forward records the context's pass count
and the backward raises if another pass has started since.  The forward
reads the pass status once (a host synchronisation), and if the tile-entry
capacity overflowed it grows the capacity and renders again.
"""
from __future__ import annotations

import torch

from . import gbr


class BlendRender(torch.autograd.Function):
    @staticmethod
    def forward(fctx, bases, weights, cams, ctx: gbr.Context):
        if bases.dim() != 3 or bases.shape[2] != 16:
            raise ValueError("bases must be [K+1, N, 16]")
        B, N = len(cams), bases.shape[1]
        bases = bases.detach().contiguous()
        weights = weights.detach().contiguous()
        raw = torch.empty(B, N, 16, device=bases.device, dtype=torch.float32)
        gbr.gbr_blend(ctx, bases, weights, raw)
        images = torch.empty(gbr.image_numel(cams), device=bases.device, dtype=torch.float32)
        offsets = [b * N for b in range(B + 1)]
        gbr.gbr_render(ctx, raw, offsets, cams, images)
        st = gbr.gbr_query_status(ctx)
        if st.overflow:
            gbr.gbr_reserve(ctx, int(st.entries * 1.25) + 1024)
            gbr.gbr_render(ctx, raw, offsets, cams, images)
            if gbr.gbr_query_status(ctx).overflow:
                raise RuntimeError("BlendRender: tile-entry overflow after growing the capacity")
        fctx.save_for_backward(bases, weights)
        fctx.gctx = ctx
        fctx.pass_id = ctx.passes
        fctx.raw = raw          # the library's backward re-reads the blended Gaussians
        return images

    @staticmethod
    def backward(fctx, dimages):
        bases, weights = fctx.saved_tensors
        if fctx.gctx.passes != fctx.pass_id:
            raise RuntimeError("BlendRender.backward: the context has rendered again since this forward; "
                               "its saved state belongs to the later pass")
        dbases = torch.empty_like(bases)
        dweights = torch.empty_like(weights)
        gbr.gbr_backward(fctx.gctx, dimages.contiguous(), bases, weights, dbases, dweights)
        return dbases, dweights, None, None


def blend_render(bases, weights, cams, ctx: gbr.Context):
    """Differentiable images (packed CHW per frame) of the blended avatars."""
    return BlendRender.apply(bases, weights, cams, ctx)
