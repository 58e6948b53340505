"""torch.autograd wrapper of transfer precompute + relight with the library's
hand-written adjoint: colour = relight(transfer(scene), light)."""
from __future__ import annotations

import torch

from . import api


class PRTGSTransfer(torch.autograd.Function):
    """colour [n, B, 3] from (means, quats, log_scales, opacity, normals, light).

    The BVH is rebuilt from the inputs on every forward (its construction is
    part of the precompute).  Direct transfer only (no bounce).  Gradients
    flow to every tensor input; the hit, hemisphere and cut-off decisions are
    held fixed (almost-everywhere gradient of the piecewise-smooth forward).
    """

    @staticmethod
    def forward(ctx, means, quats, log_scales, opacity, normals, light, params: api.TransferParams):
        if params.bounces != 0:
            raise ValueError("the adjoint covers the direct transfer only")
        scene = api.Scene(means.detach().contiguous(), quats.detach().contiguous(),
                          log_scales.detach().contiguous(), opacity.detach().contiguous(),
                          normals.detach().contiguous())
        bvh = api.build_bvh(scene)
        # the per-ray visibilities spare the adjoint one traversal per ray
        transfer, vis = api.precompute_transfer(scene, bvh, params, want_vis=True)
        colour = api.relight(transfer, light.detach())
        ctx.save_for_backward(light)
        ctx.scene, ctx.bvh, ctx.params, ctx.transfer, ctx.vis = scene, bvh, params, transfer, vis
        return colour

    @staticmethod
    def backward(ctx, d_colour):
        (light,) = ctx.saved_tensors
        dT, dL = api.relight_backward(ctx.transfer, light.detach(), d_colour,
                                      want_dT=True, want_dL=ctx.needs_input_grad[5])
        grads = api.transfer_backward(ctx.scene, ctx.bvh, ctx.params, dT, vis=ctx.vis)
        return (grads["means"], grads["quats"], grads["log_scales"], grads["opacity"], grads["normals"],
                dL.to(light.dtype) if dL is not None else None, None)


def transfer_and_relight(means, quats, log_scales, opacity, normals, light, params: api.TransferParams):
    return PRTGSTransfer.apply(means, quats, log_scales, opacity, normals, light, params)
