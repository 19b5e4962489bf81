"""torch.autograd.Function over gs_render_forward_checked /
gs_render_forward_batch / gs_render_backward.

    rgb, alpha, depth, dcdx, dcdy = rasterize(means, log_scales, quats, opacity_logits, sh, cam)

Gradients flow from rgb, alpha and depth to the five parameter tensors; the
image-gradient buffers dcdx, dcdy are outputs only (their own derivative,
a second-order term, is not formed).  The forward's workspace (sorted tile
lists, projected records) and its final_T / n_contrib buffers are the saved
state; the backward recomputes the per-tile transmittance in reverse.

Workspaces are kept between calls, per (device, Gaussian count, SH degree,
raster size), with a key capacity that only grows (half again the largest
pair count seen).  The first call of a class, and every call that will have
no backward, runs the checked forward: the host waits for the pair count
and a frame that outgrows the capacity is run again with more room.  Later
calls that build a graph do not wait: the pass is launched with the cached
capacity and its pair count is copied to pinned memory behind it; the
backward checks it before anything else, grows the capacity for the next
step when the margin shrinks, and raises GsError(GS_ERR_CAPACITY) if this
step's pairs did not fit (its outputs were then invalid and the step must
be run again; the capacity has already been grown).  A workspace returns
to the pool when the autograd graph that saved it is freed, so two graphs
alive at once never share one; every call uses the caller's current
stream, on which reuse is ordered.
"""

from __future__ import annotations

import threading

import torch

from . import abi
from . import render as R

_GROWTH = 1.5


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


def _grow(ent, needed):
    ent.capacity = max(ent.capacity, int(needed * _GROWTH) + 1024)


def _forward(ds, cam, opts, out, deferred):
    dev = ds.means.device
    key = (dev.index, ds.n, ds.sh_degree, int(cam.width), int(cam.height))
    ent = _entry(key)
    jobs = R.make_jobs([(ds, cam, opts, out)])
    if deferred and ent.capacity > 0:
        cap = ent.capacity
        L = R.layout_for(jobs, 1, cap, with_backward=True)
        ws = ent.take(L.total_bytes, dev)
        abi.check(abi.gs_render_forward_batch(jobs, 1, ws.data_ptr(), ws.numel(), cap, R.current_stream_ptr()))
        count = torch.empty(2, dtype=torch.int32, pin_memory=True)
        count.copy_(ws[L.counters:L.counters + 8].view(torch.int32), non_blocking=True)
        ev = torch.cuda.Event()
        ev.record()
        fr = R.Frame(jobs, 1, [out], ws, L, cap, None, [ds])
        return fr, _Lease(ent, ws), (ent, count, ev)
    for _ in range(4):
        cap = max(ent.capacity, 1)
        L = R.layout_for(jobs, 1, cap, with_backward=True)
        ws = ent.take(L.total_bytes, dev)
        rc, needed = R.render_checked(jobs, 1, ws, cap, with_backward=True)
        if rc == abi.GS_OK:
            if needed * _GROWTH > cap:
                _grow(ent, needed)
            return R.Frame(jobs, 1, [out], ws, L, cap, [needed], [ds]), _Lease(ent, ws), None
        ent.give(ws)
        if rc != abi.GS_ERR_CAPACITY:
            abi.check(rc)
        _grow(ent, needed)
    raise abi.GsError(abi.GS_ERR_CAPACITY, "pair count did not settle")


def _check_deferred(pending, cap):
    ent, count, ev = pending
    ev.synchronize()
    needed = int(count[0].item()) & 0xFFFFFFFF
    if needed * _GROWTH > cap:
        _grow(ent, needed)
    if needed > cap or int(count[1].item()) != 0:
        raise abi.GsError(abi.GS_ERR_CAPACITY,
                          f"this step's frame needed {needed} (tile, Gaussian) pairs, more than the cached capacity "
                          f"{cap}; its outputs were invalid.  The capacity is now {ent.capacity}: run the step "
                          "again")


class _Rasterize(torch.autograd.Function):
    @staticmethod
    def forward(ctx, means, log_scales, quats, opacity_logits, sh, cam, bg, near_z, dilation, sh_degree, deferred):
        ds = R.DeviceScene(means.detach().contiguous(), log_scales.detach().contiguous(),
                           quats.detach().contiguous(), opacity_logits.detach().contiguous(),
                           sh.detach().contiguous(), int(sh_degree))
        opts = R.opts_struct(bg, near_z, dilation)
        out = R.alloc_outputs(cam.width, cam.height, means.device)
        fr, lease, pending = _forward(ds, cam, opts, out, deferred)
        # The context keeps only the saved state (final_T, n_contrib, the
        # workspace), never the returned tensors: those hold this node as
        # their grad_fn, and a reference back to them would make a cycle that
        # only the garbage collector breaks, keeping the workspace leased.
        # The launched pass has taken the output pointers already.
        fr.outputs = [{k: out[k] for k in ("final_T", "n_contrib")}]
        for k in ("rgb", "alpha", "depth", "dcdx", "dcdy", "normal", "nv"):
            setattr(fr.jobs[0].out, k, None)
        ctx.frame = fr
        ctx.lease = lease
        ctx.pending = pending
        ctx.scene = ds
        ctx.shape = (3, int(cam.height), int(cam.width))
        ctx.mark_non_differentiable(out["dcdx"], out["dcdy"])
        return out["rgb"], out["alpha"], out["depth"], out["dcdx"], out["dcdy"]

    @staticmethod
    def backward(ctx, g_rgb, g_alpha, g_depth, _g_dcdx, _g_dcdy):
        fr = ctx.frame
        ds = ctx.scene
        # written by the adjoint (zeros included), so no clearing launches
        grads = [torch.empty_like(t) for t in ds.tensors()]
        g_rgb = (torch.zeros(ctx.shape, dtype=torch.float32, device=ds.means.device) if g_rgb is None
                 else g_rgb.contiguous().float())
        g_alpha = None if g_alpha is None else g_alpha.contiguous().float()
        g_depth = None if g_depth is None else g_depth.contiguous().float()
        R.render_backward(fr, g_rgb, grads, g_alpha, g_depth, overwrite=True)
        # the adjoint stays within the workspace whatever the pair count, so
        # it is queued first and the host waits for the forward's count while
        # the device works
        if ctx.pending is not None:
            _check_deferred(ctx.pending, fr.key_capacity)
        return (*grads, None, None, None, None, None, None)


def rasterize(means, log_scales, quats, opacity_logits, sh, cam, bg=(0.0, 0.0, 0.0), near_z=R.NEAR_Z,
              dilation=R.DILATION):
    k = sh.shape[1]
    deg = {1: 0, 4: 1, 9: 2, 16: 3}[int(k)]
    # a call that builds a graph checks its pair count in the backward
    deferred = torch.is_grad_enabled() and any(
        t.requires_grad for t in (means, log_scales, quats, opacity_logits, sh))
    return _Rasterize.apply(means, log_scales, quats, opacity_logits, sh, cam, tuple(bg), near_z, dilation, deg,
                            deferred)
