"""torch.autograd.Function around the HIP rasteriser.

forward  -> gs3_render      (the tile rasteriser of the Background section)
backward -> gs3_render_vjp  (J_img^T applied to dL/dC)
jvp      -> gs3_render_jvp  (J_img applied to a parameter tangent)

The parameters flow in as a float32 [P, N] device tensor and are copied into
the scene before each call; the per-view binning is recomputed from them.
Forward mode goes through torch.autograd.forward_ad (make_dual /
unpack_dual); reverse mode through torch.autograd.  A JVP followed by a VJP
forms the Gauss-Newton product J^T W J z of the Methodology section image by
image, which the test suite checks against gs3_hvp_diag.  (The torch.func
transforms hand a custom Function wrapper tensors without storage, which a
C ABI cannot take pointers to.)
"""
from __future__ import annotations

import torch

from .api import Scene


class RasterizeFn(torch.autograd.Function):
    """image[H, W, 3] = render(params[P, N]) for one camera of a Scene."""

    @staticmethod
    def forward(params: torch.Tensor, scene: Scene, cam: int) -> torch.Tensor:
        scene.set_params(params.detach().contiguous())
        return scene.render(cam)

    @staticmethod
    def setup_context(ctx, inputs, output):
        params, scene, cam = inputs
        ctx.scene = scene
        ctx.cam = cam
        ctx.save_for_backward(params)

    @staticmethod
    def backward(ctx, grad_img: torch.Tensor):
        (params,) = ctx.saved_tensors
        ctx.scene.set_params(params.detach().contiguous())
        g = ctx.scene.render_vjp(ctx.cam, grad_img.contiguous().float())
        return g, None, None

    @staticmethod
    def jvp(ctx, t_params: torch.Tensor, *_):
        _, tan = ctx.scene.render_jvp(ctx.cam, t_params.contiguous().float())
        return tan


def rasterize(params: torch.Tensor, scene: Scene, cam: int) -> torch.Tensor:
    return RasterizeFn.apply(params, scene, cam)
