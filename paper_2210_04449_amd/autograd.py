"""Differentiable fine SDF: vertex positions -> fine SDF through the traced rays.

`FineSDF.apply(vertices, pipeline, frames)` refits the pipeline's scene to the
given vertex positions, resets the accumulation state, runs the SDF update for
each frame index and returns the fine SDF.  Its backward calls the library's
gradient kernel (``rtsdf_trace_backward``): every texel whose value came from a
ray regenerates that ray and scatters dL/df * sign * |w| * b_i * n / (n . w) into
the three vertices of the hit triangle.  Voxelization, jump flooding,
selection, the sign and the identity of the closest ray are piecewise constant
and carry no gradient; texels that took the coarse value have none either.

Only alpha = 1 (the running minimum of Eq. (1)) is differentiated: with
alpha < 1 a texel's value can be the decayed term alpha u_{t-1} +
(1 - alpha) max(c, 0), which depends on earlier traced distances through
u_{t-1}, and the argmin record the backward follows is cleared whenever that
term wins, so the gradient would silently miss those contributions.  The
forward raises ValueError for a pipeline with alpha != 1.
"""
from __future__ import annotations

import torch

from . import rtsdf as R


class FineSDF(torch.autograd.Function):
    @staticmethod
    def forward(ctx, vertices: torch.Tensor, pipeline, frames):
        p = pipeline
        if p.alpha != 1.0:
            raise ValueError(f"FineSDF differentiates the running minimum of Eq. (1) only (alpha = 1); "
                             f"the pipeline has alpha = {p.alpha}")
        p.set_vertices(vertices.detach().to(p.device, torch.float32).contiguous())
        p.reset()
        for f in frames:
            p.step(int(f))
        ctx.pipeline = p
        ctx.version = getattr(p, "_grad_version", 0) + 1
        p._grad_version = ctx.version
        # the backward reads these; keep this forward's copies
        ctx.save_for_backward(p.fine_sdf.clone(), p.state.arg_tri.clone(), p.state.arg_ray.clone())
        return p.fine_sdf.clone()

    @staticmethod
    def backward(ctx, grad_fine: torch.Tensor):
        p = ctx.pipeline
        if getattr(p, "_grad_version", None) != ctx.version:
            raise RuntimeError("FineSDF: the pipeline ran another forward before this backward")
        fine, arg_tri, arg_ray = ctx.saved_tensors
        state = R.AccumState.wrap(p.state.u, p.state.hits, arg_tri, arg_ray)
        grad_v = torch.zeros(p.vertices.shape[0] * 3, dtype=torch.float32, device=p.device)
        R.rtsdf_trace_backward(p.scene, p.fine, state, fine, grad_fine.to(torch.float32).contiguous(), p.seed,
                               p.scene_id, grad_v)
        return grad_v.view(-1, 3), None, None


def fine_sdf(vertices: torch.Tensor, pipeline, frames) -> torch.Tensor:
    return FineSDF.apply(vertices, pipeline, frames)
