"""torch.autograd.Function over gs_render_forward_checked / gs_render_backward.

    rgb, alpha, depth, dcdx, dcdy = rasterize(means, log_scales, quats, opacity_logits, sh, cam)

Gradients flow from rgb, alpha and depth to the five parameter tensors; the
image-gradient buffers dcdx, dcdy are outputs only (their own derivative,
a second-order term, is not formed).  The forward's workspace (sorted tile
lists, projected records) and its final_T / n_contrib buffers are the saved
state; the backward recomputes the per-tile transmittance in reverse.

Workspaces are kept between calls, per (device, Gaussian count, SH degree,
raster size), with a key capacity that only grows: a step runs the checked
forward (one synchronisation on the frame's pair count, no second
projection) and, in the rare step whose pairs outgrow the capacity, grows
it by a quarter and runs again.  A workspace returns to the pool when the
autograd graph that saved it is freed, so two graphs alive at once never
share one; every call uses the caller's current stream, on which reuse is
ordered.
"""

from __future__ import annotations

import threading

import torch

from . import abi
from . import render as R

_GROWTH = 1.25


class _Entry:
    """Key capacity and idle workspaces of one (device, n, degree, W, H) class."""

    def __init__(self):
        self.capacity = 0
        self.free = []
        self.lock = threading.Lock()

    def take(self, nbytes, device):
        with self.lock:
            while self.free:
                ws = self.free.pop()
                if ws.numel() >= nbytes:
                    return ws
        return R.alloc_workspace(nbytes, device)

    def give(self, ws):
        with self.lock:
            self.free.append(ws)


_POOL: dict = {}
_POOL_LOCK = threading.Lock()


def _entry(key) -> _Entry:
    with _POOL_LOCK:
        e = _POOL.get(key)
        if e is None:
            e = _POOL[key] = _Entry()
        return e


class _Lease:
    """Hands a workspace back to its pool entry when the saving graph dies."""

    def __init__(self, entry, ws):
        self.entry, self.ws = entry, ws

    def __del__(self):
        self.entry.give(self.ws)


def _forward(ds, cam, opts, out):
    dev = ds.means.device
    key = (dev.index, ds.n, ds.sh_degree, int(cam.width), int(cam.height))
    ent = _entry(key)
    jobs = R.make_jobs([(ds, cam, opts, out)])
    for _ in range(4):
        cap = max(ent.capacity, 1)
        L = R.layout_for(jobs, 1, cap, with_backward=True)
        ws = ent.take(L.total_bytes, dev)
        rc, needed = R.render_checked(jobs, 1, ws, cap, with_backward=True)
        if rc == abi.GS_OK:
            return R.Frame(jobs, 1, [out], ws, L, cap, [needed], [ds]), _Lease(ent, ws)
        ent.give(ws)
        if rc != abi.GS_ERR_CAPACITY:
            abi.check(rc)
        ent.capacity = max(ent.capacity, int(needed * _GROWTH) + 1024)
    raise abi.GsError(abi.GS_ERR_CAPACITY, "pair count did not settle")


class _Rasterize(torch.autograd.Function):
    @staticmethod
    def forward(ctx, means, log_scales, quats, opacity_logits, sh, cam, bg, near_z, dilation, sh_degree):
        ds = R.DeviceScene(means.detach().contiguous(), log_scales.detach().contiguous(),
                           quats.detach().contiguous(), opacity_logits.detach().contiguous(),
                           sh.detach().contiguous(), int(sh_degree))
        opts = R.opts_struct(bg, near_z, dilation)
        out = R.alloc_outputs(cam.width, cam.height, means.device)
        fr, lease = _forward(ds, cam, opts, out)
        ctx.frame = fr
        ctx.lease = lease
        ctx.scene = ds
        ctx.mark_non_differentiable(out["dcdx"], out["dcdy"])
        return out["rgb"], out["alpha"], out["depth"], out["dcdx"], out["dcdy"]

    @staticmethod
    def backward(ctx, g_rgb, g_alpha, g_depth, _g_dcdx, _g_dcdy):
        fr = ctx.frame
        ds = ctx.scene
        grads = [torch.zeros_like(t) for t in ds.tensors()]
        g_rgb = torch.zeros_like(fr.outputs[0]["rgb"]) if g_rgb is None else g_rgb.contiguous().float()
        g_alpha = None if g_alpha is None else g_alpha.contiguous().float()
        g_depth = None if g_depth is None else g_depth.contiguous().float()
        R.render_backward(fr, g_rgb, grads, g_alpha, g_depth)
        return (*grads, None, None, None, None, None)


def rasterize(means, log_scales, quats, opacity_logits, sh, cam, bg=(0.0, 0.0, 0.0), near_z=R.NEAR_Z,
              dilation=R.DILATION):
    k = sh.shape[1]
    deg = {1: 0, 4: 1, 9: 2, 16: 3}[int(k)]
    return _Rasterize.apply(means, log_scales, quats, opacity_logits, sh, cam, tuple(bg), near_z, dilation, deg)
