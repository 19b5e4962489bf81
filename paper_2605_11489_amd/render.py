"""torch-facing wrapper of the C ABI: device tensors in, device tensors out.

torch only provides device memory (tensors) and streams here; every stage of
the rasterizer runs in libgs3's HIP kernels.
"""

from __future__ import annotations

import ctypes as C
import dataclasses

import numpy as np
import torch

from . import abi

NEAR_Z = 0.2
DILATION = 0.3


@dataclasses.dataclass
class DeviceScene:
    means: torch.Tensor
    log_scales: torch.Tensor
    quats: torch.Tensor
    opacity_logits: torch.Tensor
    sh: torch.Tensor
    sh_degree: int

    @property
    def n(self) -> int:
        return int(self.means.shape[0])

    @staticmethod
    def from_host(scene, device="cuda") -> "DeviceScene":
        def t(a):
            return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(device)
        return DeviceScene(t(scene.means), t(scene.log_scales), t(scene.quats), t(scene.opacity_logits),
                           t(scene.sh), int(scene.sh_degree))

    def tensors(self):
        return [self.means, self.log_scales, self.quats, self.opacity_logits, self.sh]

    def c_struct(self) -> abi.gs_scene:
        for t in self.tensors():
            if not t.is_contiguous() or t.dtype != torch.float32:
                raise ValueError("scene tensors must be contiguous float32")
        return abi.gs_scene(self.means.data_ptr(), self.log_scales.data_ptr(), self.quats.data_ptr(),
                            self.opacity_logits.data_ptr(), self.sh.data_ptr(), self.n, self.sh_degree, 0)


def camera_struct(cam) -> abi.gs_camera:
    c = abi.gs_camera()
    R = np.asarray(cam.R_wc, dtype=np.float64).reshape(9)
    t = np.asarray(cam.t, dtype=np.float64).reshape(3)
    for i in range(9):
        c.R_wc[i] = float(R[i])
    for i in range(3):
        c.t[i] = float(t[i])
    c.fx, c.fy, c.cx, c.cy = float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy)
    c.width, c.height = int(cam.width), int(cam.height)
    return c


def opts_struct(bg=(0.0, 0.0, 0.0), near_z=NEAR_Z, dilation=DILATION,
                overlap=abi.GS_OVERLAP_SQUARE) -> abi.gs_render_opts:
    o = abi.gs_render_opts()
    for i in range(3):
        o.bg[i] = float(bg[i])
    o.overlap = int(overlap)
    o.near_z = float(near_z)
    o.dilation = float(dilation)
    return o


def alloc_outputs(width: int, height: int, device="cuda", normals=False) -> dict:
    H, W = int(height), int(width)
    out = dict(rgb=torch.empty(3, H, W, device=device), alpha=torch.empty(H, W, device=device),
               depth=torch.empty(H, W, device=device), dcdx=torch.empty(3, H, W, device=device),
               dcdy=torch.empty(3, H, W, device=device), final_T=torch.empty(H, W, device=device),
               n_contrib=torch.empty(H, W, dtype=torch.int32, device=device))
    if normals:
        out["normal"] = torch.empty(3, H, W, device=device)
        out["nv"] = torch.empty(H, W, device=device)
    return out


def outputs_struct(out: dict) -> abi.gs_outputs:
    def p(name):
        t = out.get(name)
        return None if t is None else t.data_ptr()
    return abi.gs_outputs(p("rgb"), p("alpha"), p("depth"), p("dcdx"), p("dcdy"), p("final_T"), p("n_contrib"),
                          p("n_evaluated"), p("n_blended"), p("normal"), p("nv"))


def current_stream_ptr():
    return torch.cuda.current_stream().cuda_stream


def alloc_workspace(nbytes: int, device="cuda") -> torch.Tensor:
    ws = torch.empty(max(int(nbytes), 256) + 256, dtype=torch.uint8, device=device)
    off = (-ws.data_ptr()) % 256
    return ws[off:off + max(int(nbytes), 256)]


@dataclasses.dataclass
class Frame:
    jobs: object                 # ctypes gs_job array (kept alive)
    n_jobs: int
    outputs: list                # per job dict of tensors
    workspace: torch.Tensor
    layout: abi.gs_ws_layout
    key_capacity: int
    keys_per_job: list
    holders: list                # scenes kept alive while the frame is in flight


def make_jobs(items):
    """items: list of (DeviceScene, camera, opts_struct, outputs dict)."""
    arr = (abi.gs_job * len(items))()
    for i, (sc, cam, op, out) in enumerate(items):
        arr[i].scene = sc.c_struct()
        arr[i].cam = camera_struct(cam) if not isinstance(cam, abi.gs_camera) else cam
        arr[i].opts = op
        arr[i].out = outputs_struct(out) if out is not None else abi.gs_outputs()
    return arr


def layout_for(jobs, n_jobs, key_capacity, with_backward=False) -> abi.gs_ws_layout:
    L = abi.gs_ws_layout()
    abi.check(abi.gs_forward_layout(jobs, n_jobs, int(key_capacity), int(bool(with_backward)), C.byref(L)))
    return L


def count_keys(jobs, n_jobs, device="cuda") -> list:
    L = layout_for(jobs, n_jobs, 0)
    ws = alloc_workspace(L.total_bytes, device)
    keys = (C.c_int64 * n_jobs)()
    abi.check(abi.gs_count_keys(jobs, n_jobs, ws.data_ptr(), ws.numel(), keys, current_stream_ptr()))
    return [int(k) for k in keys]


def render_batch(items, key_capacity=None, with_backward=False, device="cuda", headroom=1.0,
                 workspace=None) -> Frame:
    jobs = make_jobs(items)
    n = len(items)
    kpj = None
    if key_capacity is None:
        kpj = count_keys(jobs, n, device)
        key_capacity = max(1, int(sum(kpj) * headroom))
    L = layout_for(jobs, n, key_capacity, with_backward)
    ws = workspace if workspace is not None and workspace.numel() >= L.total_bytes else alloc_workspace(L.total_bytes, device)
    abi.check(abi.gs_render_forward_batch(jobs, n, ws.data_ptr(), ws.numel(), int(key_capacity),
                                          current_stream_ptr()))
    return Frame(jobs, n, [it[3] for it in items], ws, L, int(key_capacity), kpj, [it[0] for it in items])


def render(scene: DeviceScene, cam, bg=(0.0, 0.0, 0.0), near_z=NEAR_Z, dilation=DILATION, key_capacity=None,
           with_backward=False, device="cuda", normals=False) -> Frame:
    out = alloc_outputs(cam.width, cam.height, device, normals=normals)
    return render_batch([(scene, cam, opts_struct(bg, near_z, dilation), out)], key_capacity, with_backward,
                        device)


def forward_status(frame: Frame):
    """(return code, keys the frame needed); synchronises the device."""
    torch.cuda.synchronize()
    k = C.c_int64(0)
    rc = abi.gs_forward_status(frame.workspace.data_ptr(), C.byref(frame.layout), C.byref(k))
    return rc, int(k.value)


def sorted_keys(frame: Frame, job: int = 0, count=None):
    """Sorted (tile << 32 | z bits) keys and local Gaussian indices of one job,
    as numpy uint64 / uint32 arrays."""
    if count is None:
        if frame.keys_per_job is None:
            frame.keys_per_job = count_keys(frame.jobs, frame.n_jobs, frame.workspace.device)
        count = frame.keys_per_job[job]
    dev = frame.workspace.device
    cap = max(count, frame.key_capacity, 1)   # room for every pair the workspace can hold
    keys = torch.empty(cap, dtype=torch.int64, device=dev)
    vals = torch.empty(cap, dtype=torch.int32, device=dev)
    abi.check(abi.gs_sorted_keys(frame.jobs, frame.n_jobs, job, frame.workspace.data_ptr(), C.byref(frame.layout),
                                 keys.data_ptr(), vals.data_ptr(), current_stream_ptr()))
    torch.cuda.synchronize()
    return (keys[:count].cpu().numpy().view(np.uint64), vals[:count].cpu().numpy().view(np.uint32))


def render_backward(frame: Frame, g_rgb, grads, g_alpha=None, g_depth=None, overwrite=False):
    """gs_render_backward over a one-frame Frame rendered with
    with_backward=True (its scene, camera, options and outputs): accumulates
    (+=) into the five tensors `grads` (shapes of the scene's tensors), or
    writes them when `overwrite`, on the current stream."""
    if frame.n_jobs != 1:
        raise ValueError("the backward pass takes a one-frame workspace")
    for t in (g_rgb, g_alpha, g_depth):
        if t is not None and not (t.is_contiguous() and t.dtype == torch.float32):
            raise ValueError("loss gradients must be contiguous float32")
    gs = abi.gs_grads(*[g.data_ptr() for g in grads], int(bool(overwrite)), 0)
    j = frame.jobs[0]
    sc, cs, opts, outs = j.scene, j.cam, j.opts, j.out
    abi.check(abi.gs_render_backward(C.byref(sc), C.byref(cs), C.byref(opts), C.byref(outs),
                                     frame.workspace.data_ptr(), frame.workspace.numel(), frame.key_capacity,
                                     g_rgb.data_ptr(), None if g_alpha is None else g_alpha.data_ptr(),
                                     None if g_depth is None else g_depth.data_ptr(), C.byref(gs),
                                     current_stream_ptr()))


def render_checked(jobs, n_jobs, workspace, key_capacity, with_backward=False):
    """gs_render_forward_checked: (return code, pairs the frame needs)."""
    k = C.c_int64(0)
    rc = abi.gs_render_forward_checked(jobs, n_jobs, workspace.data_ptr(), workspace.numel(), int(key_capacity),
                                       int(bool(with_backward)), C.byref(k), current_stream_ptr())
    return rc, int(k.value)


def workspace_view(frame: Frame, region: str, dtype, count: int):
    off = getattr(frame.layout, region)
    itemsize = torch.empty(0, dtype=dtype).element_size()
    return frame.workspace[off:off + count * itemsize].view(dtype)


def gradient_upsample(rgb, dcdx, dcdy, scale: int):
    """Gradient-aware interpolation (Sec. 4.1, Eq. 5-7) of planar [3, H, W]
    float32 device tensors to [3, H*scale, W*scale], on the current stream."""
    for t in (rgb, dcdx, dcdy):
        if not (t.is_cuda and t.dtype == torch.float32 and t.is_contiguous() and t.shape == rgb.shape):
            raise ValueError("rgb, dcdx, dcdy must be contiguous float32 device tensors of one shape [3, H, W]")
    _, H, W = rgb.shape
    out = torch.empty(3, H * scale, W * scale, dtype=torch.float32, device=rgb.device)
    abi.check(abi.gs_gradient_upsample(rgb.data_ptr(), dcdx.data_ptr(), dcdy.data_ptr(), W, H, scale,
                                       out.data_ptr(), current_stream_ptr()))
    return out


def warp_workspace_bytes(src_cam, dst_cam) -> int:
    n = C.c_size_t(0)
    abi.check(abi.gs_warp_workspace_size(C.byref(camera_struct(src_cam)), C.byref(camera_struct(dst_cam)),
                                         C.byref(n)))
    return int(n.value)


def motion_warp(src_cam, dst_cam, rgb, alpha, depth, dcdx, dcdy, workspace=None, out=None, normal=None):
    """Motion vectors (Sec. 4.2, Eq. 12) of a frame rendered from `src_cam`
    and its forward warp (Eq. 13) to `dst_cam`, on the current stream.
    alpha, depth: [H, W] float32 device tensors (required); rgb, dcdx, dcdy
    and normal: planar [3, H, W] or None (that output is then not formed;
    dcdx and dcdy go together).  Returns a dict of device tensors: motion
    [2, H, W], depth, weight [H', W'], source [H', W'] int32, and rgb, dcdx,
    dcdy, normal [3, H', W'] for the inputs given (written into `out` when
    it is such a dict)."""
    H, W = int(src_cam.height), int(src_cam.width)
    Hd, Wd = int(dst_cam.height), int(dst_cam.width)
    planes = dict(rgb=rgb, dcdx=dcdx, dcdy=dcdy, normal=normal)
    for name, t, shape in (("alpha", alpha, (H, W)), ("depth", depth, (H, W)),
                           *((k, v, (3, H, W)) for k, v in planes.items() if v is not None)):
        if not (t.is_cuda and t.dtype == torch.float32 and t.is_contiguous() and tuple(t.shape) == shape):
            raise ValueError(f"{name} must be a contiguous float32 device tensor of shape {shape}")
    if (dcdx is None) != (dcdy is None):
        raise ValueError("dcdx and dcdy go together")
    if out is None:
        out = alloc_warp_outputs(W, H, Wd, Hd, alpha.device, planes=[k for k, v in planes.items() if v is not None])
    nbytes = warp_workspace_bytes(src_cam, dst_cam)
    if workspace is None:
        workspace = alloc_workspace(nbytes, device=alpha.device)

    def p(t):
        return None if t is None else t.data_ptr()

    o = abi.gs_warp_outputs(*(p(out.get(k)) for k in ("rgb", "depth", "dcdx", "dcdy", "weight", "source",
                                                      "normal")))
    abi.check(abi.gs_motion_warp(C.byref(camera_struct(src_cam)), C.byref(camera_struct(dst_cam)), p(rgb),
                                 alpha.data_ptr(), depth.data_ptr(), p(dcdx), p(dcdy), p(normal),
                                 out["motion"].data_ptr(), C.byref(o), workspace.data_ptr(),
                                 workspace.numel() * workspace.element_size(), current_stream_ptr()))
    return out


def alloc_warp_outputs(width, height, dst_width, dst_height, device="cuda",
                       planes=("rgb", "dcdx", "dcdy")) -> dict:
    f = dict(dtype=torch.float32, device=device)
    H, W, Hd, Wd = height, width, dst_height, dst_width
    out = dict(motion=torch.empty(2, H, W, **f), depth=torch.empty(Hd, Wd, **f), weight=torch.empty(Hd, Wd, **f),
               source=torch.empty(Hd, Wd, dtype=torch.int32, device=device))
    for k in planes:
        out[k] = torch.empty(3, Hd, Wd, **f)
    return out
