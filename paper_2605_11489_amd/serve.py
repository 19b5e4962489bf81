"""Python handle on the C ABI's continuous-batching server (gs_server_*).

Marshalling only: admission, batching, memory accounting and the launches
all happen in libgs3's worker thread.
"""

from __future__ import annotations

import ctypes as C

import torch

from . import abi
from . import render as R


class _DevArray:
    """Exposes a device pointer to torch through __cuda_array_interface__."""

    def __init__(self, ptr, shape, typestr):
        self.__cuda_array_interface__ = {"shape": tuple(shape), "typestr": typestr, "data": (int(ptr), False),
                                         "version": 3, "strides": None}


_hip = None


def _hip_runtime():
    global _hip
    if _hip is None:
        _hip = C.CDLL("libamdhip64.so")    # the runtime torch already loaded
        _hip.hipMemcpy.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t, C.c_int]
        _hip.hipMemcpy.restype = C.c_int
    return _hip


def device_view(ptr, shape, dtype=torch.float32):
    """A tensor over server memory (zero copy when torch accepts
    __cuda_array_interface__, else a device-to-device copy)."""
    typestr = {torch.float32: "<f4", torch.int32: "<i4"}[dtype]
    try:
        return torch.as_tensor(_DevArray(ptr, shape, typestr), device="cuda")
    except (TypeError, RuntimeError, ValueError):
        out = torch.empty(shape, dtype=dtype, device="cuda")
        torch.cuda.synchronize()
        rc = _hip_runtime().hipMemcpy(out.data_ptr(), int(ptr), out.numel() * out.element_size(), 3)
        if rc != 0:
            raise RuntimeError(f"hipMemcpy failed with {rc}")
        return out


class Server:
    def __init__(self, budget_bytes: int, max_batch: int = 16, queue_depth: int = 4096, n_streams: int = 2,
                 fifo: bool = False, key_factor: float = 1.5, simulate: bool = False, sim_fail_every: int = 0,
                 sim_batch_us: float = 500.0, heavy_ms: float = 0.6, work_queue: bool = False):
        o = abi.gs_server_opts(int(budget_bytes), int(max_batch), int(queue_depth), int(n_streams), int(bool(fifo)),
                               float(key_factor), int(bool(simulate)), int(sim_fail_every), float(sim_batch_us),
                               float(heavy_ms), int(bool(work_queue)))
        h = C.c_void_p()
        abi.check(abi.gs_server_create(C.byref(o), C.byref(h)))
        self.h = h
        self.simulate = simulate

    def close(self):
        if self.h:
            abi.check(abi.gs_server_destroy(self.h))
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def register(self, scene) -> int:
        """scene: DeviceScene (or, when simulating, anything with n and sh_degree)."""
        if self.simulate and not isinstance(scene, R.DeviceScene):
            s = abi.gs_scene(256, 256, 256, 256, 256, int(scene.n), int(scene.sh_degree), 0)
        else:
            s = scene.c_struct()
        sid = C.c_int32(0)
        abi.check(abi.gs_scene_register(self.h, C.byref(s), C.byref(sid)))
        return int(sid.value)

    def submit_rc(self, scene_id, cam, bg=(0.0, 0.0, 0.0), near_z=R.NEAR_Z, dilation=R.DILATION):
        """(return code, ticket)."""
        t = C.c_uint64(0)
        c = R.camera_struct(cam) if not isinstance(cam, abi.gs_camera) else cam
        o = R.opts_struct(bg, near_z, dilation)
        rc = abi.gs_submit(self.h, int(scene_id), C.byref(c), C.byref(o), C.byref(t))
        return rc, int(t.value)

    def submit(self, scene_id, cam, **kw) -> int:
        rc, t = self.submit_rc(scene_id, cam, **kw)
        abi.check(rc)
        return t

    def poll(self, ticket):
        """None while in flight, else a gs_result."""
        r = abi.gs_result()
        rc = abi.gs_poll(self.h, C.c_uint64(ticket), C.byref(r))
        if rc == abi.GS_ERR_NOT_READY:
            return None
        abi.check(rc)
        return r

    def outputs(self, res) -> dict:
        """Device tensors viewing a finished request's outputs (valid until release)."""
        H, W = res.height, res.width
        o = res.out
        return dict(rgb=device_view(o.rgb, (3, H, W)), alpha=device_view(o.alpha, (H, W)),
                    depth=device_view(o.depth, (H, W)), dcdx=device_view(o.dcdx, (3, H, W)),
                    dcdy=device_view(o.dcdy, (3, H, W)), final_T=device_view(o.final_T, (H, W)),
                    n_contrib=device_view(o.n_contrib, (H, W), torch.int32))

    def release(self, ticket):
        abi.check(abi.gs_release(self.h, C.c_uint64(ticket)))

    def stats(self) -> dict:
        st = (C.c_int64 * 9)()
        abi.check(abi.gs_server_stats(self.h, st))
        keys = ("submitted", "completed", "failed", "rejected", "batches", "max_batch", "bytes_in_use", "bytes_peak",
                "flag_done")
        return dict(zip(keys, [int(v) for v in st]))
