"""torch.autograd.Function over the HIP render and its hand-written adjoint."""
from __future__ import annotations

import torch

from .raster import GaussianTensors, Plan, PlaneTensors


class RenderPlanesFn(torch.autograd.Function):
    """image = render(means, lraw, intensity, opacity; planes).

    Gradients flow to the four Gaussian tensors (the paper optimises only
    the Gaussians, Section 4.5); plane poses are inputs without gradient.
    """

    @staticmethod
    def forward(ctx, means, lraw, intensity, opacity, rot, origin, spacing, plan: Plan):
        g = GaussianTensors(means.detach(), lraw.detach(), intensity.detach(), opacity.detach())
        pl = PlaneTensors(rot.detach(), origin.detach(), spacing.detach())
        image = plan.render(g, pl)
        ctx.plan = plan
        ctx.fwd_id = plan.forward_count
        ctx.save_for_backward(means, lraw, intensity, opacity, rot, origin, spacing, image)
        return image

    @staticmethod
    def backward(ctx, d_image):
        plan: Plan = ctx.plan
        if plan.forward_count != ctx.fwd_id:
            raise RuntimeError("the plan rendered again before this backward: its workspace no longer holds "
                               "this forward's state (use one plan per pending backward)")
        means, lraw, intensity, opacity, rot, origin, spacing, image = ctx.saved_tensors
        g = GaussianTensors(means, lraw, intensity, opacity)
        pl = PlaneTensors(rot, origin, spacing)
        grads = plan.backward(g, pl, image, d_image)
        return grads.means, grads.lraw, grads.intensity, grads.opacity, None, None, None, None


def render_planes(g: GaussianTensors, planes: PlaneTensors, plan: Plan) -> torch.Tensor:
    """Differentiable render of all planes of ``plan`` (packed image)."""
    return RenderPlanesFn.apply(g.means, g.lraw, g.intensity, g.opacity, planes.rot, planes.origin,
                                planes.spacing, plan)
