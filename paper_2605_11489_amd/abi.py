"""ctypes binding of libgs3 (include/gs3.h): the same entry points under the
same names, argument marshalling only.  Every step of the rasterizer runs in
the library's HIP kernels; this module converts Python objects to the C
structs and checks return codes.

torch is imported before the library is loaded so that the process uses one
HIP runtime (the one torch already mapped).  A missing library raises
immediately: there is no fallback path.
"""

from __future__ import annotations

import ctypes as C
import os

import torch  # noqa: F401  (loads the HIP runtime first)

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgs3.so")

GS_OK = 0
GS_ERR_INVALID_ARG = -1
GS_ERR_OOM = -2
GS_ERR_TOO_LARGE = -3
GS_ERR_AGAIN = -4
GS_ERR_NOT_READY = -5
GS_ERR_HIP = -6
GS_ERR_CAPACITY = -7
GS_ERR_NOT_FOUND = -8
GS_MAX_BATCH = 64

ERR_NAMES = {0: "GS_OK", -1: "GS_ERR_INVALID_ARG", -2: "GS_ERR_OOM", -3: "GS_ERR_TOO_LARGE",
             -4: "GS_ERR_AGAIN", -5: "GS_ERR_NOT_READY", -6: "GS_ERR_HIP", -7: "GS_ERR_CAPACITY",
             -8: "GS_ERR_NOT_FOUND"}


class GsError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERR_NAMES.get(code, code)}: {msg}")
        self.code = code


class gs_scene(C.Structure):
    _fields_ = [("means", C.c_void_p), ("log_scales", C.c_void_p), ("quats", C.c_void_p),
                ("opacity_logits", C.c_void_p), ("sh", C.c_void_p), ("n", C.c_int64),
                ("sh_degree", C.c_int32), ("reserved", C.c_int32)]


class gs_camera(C.Structure):
    _fields_ = [("R_wc", C.c_double * 9), ("t", C.c_double * 3), ("fx", C.c_double), ("fy", C.c_double),
                ("cx", C.c_double), ("cy", C.c_double), ("width", C.c_int32), ("height", C.c_int32)]


GS_OVERLAP_SQUARE = 0
GS_OVERLAP_OPACITY = 1
GS_OVERLAP_ELLIPSE = 2


class gs_render_opts(C.Structure):
    _fields_ = [("bg", C.c_float * 3), ("overlap", C.c_int32), ("near_z", C.c_double),
                ("dilation", C.c_double)]


class gs_outputs(C.Structure):
    _fields_ = [("rgb", C.c_void_p), ("alpha", C.c_void_p), ("depth", C.c_void_p), ("dcdx", C.c_void_p),
                ("dcdy", C.c_void_p), ("final_T", C.c_void_p), ("n_contrib", C.c_void_p),
                ("n_evaluated", C.c_void_p), ("n_blended", C.c_void_p), ("normal", C.c_void_p),
                ("nv", C.c_void_p)]


class gs_grads(C.Structure):
    _fields_ = [("means", C.c_void_p), ("log_scales", C.c_void_p), ("quats", C.c_void_p),
                ("opacity_logits", C.c_void_p), ("sh", C.c_void_p), ("overwrite", C.c_int32),
                ("reserved", C.c_int32)]


class gs_job(C.Structure):
    _fields_ = [("scene", gs_scene), ("cam", gs_camera), ("opts", gs_render_opts), ("out", gs_outputs)]


class gs_ws_layout(C.Structure):
    _fields_ = [("total_bytes", C.c_size_t), ("n_flat", C.c_int64), ("n_tiles", C.c_int64),
                ("key_capacity", C.c_int64), ("records", C.c_size_t), ("depth_keys", C.c_size_t),
                ("rects", C.c_size_t), ("touched", C.c_size_t), ("depth_order", C.c_size_t),
                ("depth_rects", C.c_size_t),
                ("chunk_counts", C.c_size_t), ("tile_keys", C.c_size_t), ("tile_values", C.c_size_t),
                ("ranges", C.c_size_t), ("counters", C.c_size_t), ("grads2d", C.c_size_t),
                ("normals", C.c_size_t),
                ("gauss_base", C.c_int64 * GS_MAX_BATCH), ("tile_base", C.c_int64 * GS_MAX_BATCH)]


class gs_server_opts(C.Structure):
    _fields_ = [("hbm_budget_bytes", C.c_size_t), ("max_batch", C.c_int32), ("queue_depth", C.c_int32),
                ("n_streams", C.c_int32), ("fifo", C.c_int32), ("key_factor", C.c_double),
                ("simulate", C.c_int32), ("sim_fail_every", C.c_int32), ("sim_batch_us", C.c_double),
                ("heavy_ms", C.c_double), ("work_queue", C.c_int32)]


class gs_result(C.Structure):
    _fields_ = [("status", C.c_int32), ("width", C.c_int32), ("height", C.c_int32), ("batch_size", C.c_int32),
                ("retries", C.c_int32), ("flag_done", C.c_int32), ("out", gs_outputs), ("t_submit", C.c_double), ("t_start", C.c_double),
                ("t_done", C.c_double)]


class gs_warp_outputs(C.Structure):
    _fields_ = [("rgb", C.c_void_p), ("depth", C.c_void_p), ("dcdx", C.c_void_p), ("dcdy", C.c_void_p),
                ("weight", C.c_void_p), ("source", C.c_void_p), ("normal", C.c_void_p)]


P = C.POINTER
_SIGNATURES = {
    "gs_forward_layout": (C.c_int, [P(gs_job), C.c_int, C.c_int64, C.c_int, P(gs_ws_layout)]),
    "gs_count_keys": (C.c_int, [P(gs_job), C.c_int, C.c_void_p, C.c_size_t, P(C.c_int64), C.c_void_p]),
    "gs_render_forward_batch": (C.c_int, [P(gs_job), C.c_int, C.c_void_p, C.c_size_t, C.c_int64, C.c_void_p]),
    "gs_render_forward_checked": (C.c_int, [P(gs_job), C.c_int, C.c_void_p, C.c_size_t, C.c_int64, C.c_int,
                                            P(C.c_int64), C.c_void_p]),
    "gs_render_forward_noalloc": (C.c_int, [P(gs_job), C.c_int, C.c_int64, C.c_void_p, C.c_void_p]),
    "gs_render_forward": (C.c_int, [P(gs_scene), P(gs_camera), P(gs_render_opts), P(gs_outputs), C.c_void_p,
                                    C.c_size_t, C.c_int64, C.c_void_p]),
    "gs_forward_status": (C.c_int, [C.c_void_p, P(gs_ws_layout), P(C.c_int64)]),
    "gs_sorted_keys": (C.c_int, [P(gs_job), C.c_int, C.c_int, C.c_void_p, P(gs_ws_layout), C.c_void_p,
                                 C.c_void_p, C.c_void_p]),
    "gs_render_backward": (C.c_int, [P(gs_scene), P(gs_camera), P(gs_render_opts), P(gs_outputs), C.c_void_p,
                                     C.c_size_t, C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p, P(gs_grads),
                                     C.c_void_p]),
    "gs_server_create": (C.c_int, [P(gs_server_opts), P(C.c_void_p)]),
    "gs_server_destroy": (C.c_int, [C.c_void_p]),
    "gs_scene_register": (C.c_int, [C.c_void_p, P(gs_scene), P(C.c_int32)]),
    "gs_submit": (C.c_int, [C.c_void_p, C.c_int32, P(gs_camera), P(gs_render_opts), P(C.c_uint64)]),
    "gs_poll": (C.c_int, [C.c_void_p, C.c_uint64, P(gs_result)]),
    "gs_release": (C.c_int, [C.c_void_p, C.c_uint64]),
    "gs_server_stats": (C.c_int, [C.c_void_p, P(C.c_int64)]),
    "gs_gradient_upsample": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_int32, C.c_int32,
                                       C.c_void_p, C.c_void_p]),
    "gs_warp_workspace_size": (C.c_int, [P(gs_camera), P(gs_camera), P(C.c_size_t)]),
    "gs_motion_warp": (C.c_int, [P(gs_camera), P(gs_camera), C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                 C.c_void_p, C.c_void_p, C.c_void_p, P(gs_warp_outputs), C.c_void_p, C.c_size_t,
                                 C.c_void_p]),
    "gs_profile_start": (C.c_int, [C.c_int, C.c_int]),
    "gs_profile_stop": (C.c_int, [P(C.c_double), P(C.c_int64)]),
    "gs_last_error": (C.c_char_p, []),
}

_lib = None


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2605_11489_amd.build` (there is no fallback)")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGNATURES.items():
            if hasattr(L, name):
                f = getattr(L, name)
                f.restype = res
                f.argtypes = args
        _lib = L
    return _lib


def check(rc):
    if rc != GS_OK:
        msg = lib().gs_last_error()
        raise GsError(rc, msg.decode() if msg else "")
    return rc


def last_error() -> str:
    m = lib().gs_last_error()
    return m.decode() if m else ""


def _call(name, *args):
    return getattr(lib(), name)(*args)


# same names as the C entry points
def gs_forward_layout(jobs, n_jobs, key_capacity, with_backward, layout):
    return _call("gs_forward_layout", jobs, n_jobs, key_capacity, with_backward, layout)


def gs_count_keys(jobs, n_jobs, workspace, ws_bytes, keys_per_job, stream):
    return _call("gs_count_keys", jobs, n_jobs, workspace, ws_bytes, keys_per_job, stream)


def gs_render_forward_batch(jobs, n_jobs, workspace, ws_bytes, key_capacity, stream):
    return _call("gs_render_forward_batch", jobs, n_jobs, workspace, ws_bytes, key_capacity, stream)


def gs_render_forward_checked(jobs, n_jobs, workspace, ws_bytes, key_capacity, with_backward, keys_needed, stream):
    return _call("gs_render_forward_checked", jobs, n_jobs, workspace, ws_bytes, key_capacity, with_backward,
                 keys_needed, stream)


def gs_render_forward_noalloc(jobs, n_jobs, key_capacity, counts_out, stream):
    return _call("gs_render_forward_noalloc", jobs, n_jobs, key_capacity, counts_out, stream)


def gs_render_forward(scene, cam, opts, out, workspace, ws_bytes, key_capacity, stream):
    return _call("gs_render_forward", scene, cam, opts, out, workspace, ws_bytes, key_capacity, stream)


def gs_forward_status(workspace, layout, keys_needed):
    return _call("gs_forward_status", workspace, layout, keys_needed)


def gs_sorted_keys(jobs, n_jobs, job, workspace, layout, keys_out, values_out, stream):
    return _call("gs_sorted_keys", jobs, n_jobs, job, workspace, layout, keys_out, values_out, stream)


def gs_render_backward(scene, cam, opts, fwd_out, workspace, ws_bytes, key_capacity, dl_drgb, dl_dalpha,
                       dl_ddepth, grads, stream):
    return _call("gs_render_backward", scene, cam, opts, fwd_out, workspace, ws_bytes, key_capacity, dl_drgb,
                 dl_dalpha, dl_ddepth, grads, stream)


def gs_server_create(opts, server):
    return _call("gs_server_create", opts, server)


def gs_server_destroy(server):
    return _call("gs_server_destroy", server)


def gs_scene_register(server, scene, scene_id):
    return _call("gs_scene_register", server, scene, scene_id)


def gs_submit(server, scene_id, cam, opts, ticket):
    return _call("gs_submit", server, scene_id, cam, opts, ticket)


def gs_poll(server, ticket, result):
    return _call("gs_poll", server, ticket, result)


def gs_release(server, ticket):
    return _call("gs_release", server, ticket)


def gs_server_stats(server, stats):
    return _call("gs_server_stats", server, stats)


def gs_gradient_upsample(rgb, dcdx, dcdy, width, height, scale, out, stream):
    return _call("gs_gradient_upsample", rgb, dcdx, dcdy, width, height, scale, out, stream)


def gs_warp_workspace_size(src, dst, nbytes):
    return _call("gs_warp_workspace_size", src, dst, nbytes)


def gs_motion_warp(src, dst, rgb, alpha, depth, dcdx, dcdy, normal, motion, out, workspace, ws_bytes, stream):
    return _call("gs_motion_warp", src, dst, rgb, alpha, depth, dcdx, dcdy, normal, motion, out, workspace,
                 ws_bytes, stream)


def gs_profile_start(max_frames, every=1):
    return _call("gs_profile_start", max_frames, every)


def gs_profile_stop(stage_ms, frames):
    return _call("gs_profile_stop", stage_ms, frames)


GS_N_STAGES = 5
STAGE_NAMES = ("project", "depth_sort", "emit", "tile_sort", "composite")


def gs_last_error():
    return _call("gs_last_error")
