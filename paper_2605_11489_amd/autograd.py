"""torch.autograd.Function over gs_render_forward / gs_render_backward.

    rgb, alpha, depth, dcdx, dcdy = rasterize(means, log_scales, quats, opacity_logits, sh, cam)

Gradients flow from rgb, alpha and depth to the five parameter tensors; the
image-gradient buffers dcdx, dcdy are outputs only (their own derivative,
a second-order term, is not formed).  The forward's workspace (sorted tile
lists, projected records) and its final_T / n_contrib buffers are the saved
state; the backward recomputes the per-tile transmittance in reverse.
"""

from __future__ import annotations

import ctypes as C

import torch

from . import abi
from . import render as R


class _Rasterize(torch.autograd.Function):
    @staticmethod
    def forward(ctx, means, log_scales, quats, opacity_logits, sh, cam, bg, near_z, dilation, sh_degree):
        ds = R.DeviceScene(means.detach().contiguous(), log_scales.detach().contiguous(),
                           quats.detach().contiguous(), opacity_logits.detach().contiguous(),
                           sh.detach().contiguous(), int(sh_degree))
        fr = R.render(ds, cam, bg=bg, near_z=near_z, dilation=dilation, with_backward=True,
                      device=means.device)
        out = fr.outputs[0]
        ctx.frame = fr
        ctx.scene = ds
        ctx.cam = cam
        ctx.opts = (bg, near_z, dilation)
        ctx.mark_non_differentiable(out["dcdx"], out["dcdy"])
        return out["rgb"], out["alpha"], out["depth"], out["dcdx"], out["dcdy"]

    @staticmethod
    def backward(ctx, g_rgb, g_alpha, g_depth, _g_dcdx, _g_dcdy):
        fr = ctx.frame
        ds = ctx.scene
        bg, near_z, dilation = ctx.opts
        dev = ds.means.device
        grads = [torch.zeros_like(t) for t in ds.tensors()]
        g_rgb = torch.zeros_like(fr.outputs[0]["rgb"]) if g_rgb is None else g_rgb.contiguous().float()
        g_alpha = None if g_alpha is None else g_alpha.contiguous().float()
        g_depth = None if g_depth is None else g_depth.contiguous().float()
        gs = abi.gs_grads(*[g.data_ptr() for g in grads])
        scene = ds.c_struct()
        cam = R.camera_struct(ctx.cam)
        opts = R.opts_struct(bg, near_z, dilation)
        outs = R.outputs_struct(fr.outputs[0])
        abi.check(abi.gs_render_backward(C.byref(scene), C.byref(cam), C.byref(opts), C.byref(outs),
                                         fr.workspace.data_ptr(), fr.workspace.numel(), fr.key_capacity,
                                         g_rgb.data_ptr(), None if g_alpha is None else g_alpha.data_ptr(),
                                         None if g_depth is None else g_depth.data_ptr(), C.byref(gs),
                                         R.current_stream_ptr()))
        del dev
        return (*grads, None, None, None, None, None)


def rasterize(means, log_scales, quats, opacity_logits, sh, cam, bg=(0.0, 0.0, 0.0), near_z=R.NEAR_Z,
              dilation=R.DILATION):
    k = sh.shape[1]
    deg = {1: 0, 4: 1, 9: 2, 16: 3}[int(k)]
    return _Rasterize.apply(means, log_scales, quats, opacity_logits, sh, cam, tuple(bg), near_z, dilation, deg)
