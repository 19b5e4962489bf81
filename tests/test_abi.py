"""The C ABI on the CPU: the library loads, exports every entry point that
include/gs3.h declares, and its host-only calls (layout planning, argument
checks) behave as documented.  No kernel is launched."""

import ctypes as C
import os
import re

import pytest

import synth

torch = pytest.importorskip("torch")
from paper_2605_11489_amd import abi  # noqa: E402
from paper_2605_11489_amd import render as R  # noqa: E402

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared():
    names = []
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            src = open(os.path.join(ROOT, "include", fn)).read()
            names += re.findall(r"^(?:int|const char\*|void)\s+(gs_\w+)\s*\(", src, re.M)
    return sorted(set(names))


def test_library_exports_every_declared_symbol():
    lib = abi.lib()
    names = declared()
    assert len(names) >= 10
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_has_same_names():
    for n in declared():
        assert hasattr(abi, n), n


def fake_job(n=1000, W=960, H=540, deg=3):
    j = (abi.gs_job * 1)()
    j[0].scene = abi.gs_scene(256, 256, 256, 256, 256, n, deg, 0)
    j[0].cam = R.camera_struct(synth.cfg2_camera(W, H))
    j[0].opts = R.opts_struct()
    return j


def test_layout_regions_are_aligned_and_disjoint():
    j = fake_job(1_000_000)
    L = R.layout_for(j, 1, 11_000_000, with_backward=True)
    assert L.n_tiles == 60 * 34 and L.n_flat == 1_000_192
    regions = [("records", 48 * L.n_flat), ("depth_keys", 4 * L.n_flat), ("rects", 4 * L.n_flat),
               ("touched", 4 * L.n_flat), ("depth_order", 4 * L.n_flat), ("depth_rects", 4 * L.n_flat),
               ("chunk_counts", 4 * (-(-L.n_flat // 256) - (-L.n_flat // 4096) + 2)),
               ("tile_keys", 4 * L.key_capacity), ("tile_values", 4 * L.key_capacity),
               ("ranges", 8 * L.n_tiles), ("counters", 576), ("grads2d", 40 * L.n_flat)]
    spans = sorted((getattr(L, r), getattr(L, r) + sz, r) for r, sz in regions)
    for (a0, a1, ra), (b0, b1, rb) in zip(spans, spans[1:]):
        assert a1 <= b0, (ra, rb)
    for a0, a1, r in spans:
        assert a0 % 256 == 0, r
    assert spans[-1][1] <= L.total_bytes
    L2 = R.layout_for(j, 1, 11_000_000, with_backward=False)
    assert L2.total_bytes < L.total_bytes and L2.tile_values == L.tile_values
    assert L.normals == 0 and L2.normals == 0


def test_layout_normals_region():
    """Asking a frame for normal or nv outputs adds a 16 B per Gaussian
    region after the public ones; nothing before it moves."""
    j = fake_job(1_000_000)
    L0 = R.layout_for(j, 1, 11_000_000)
    for field in ("normal", "nv"):
        jn = fake_job(1_000_000)
        setattr(jn[0].out, field, 1 << 20)
        L = R.layout_for(jn, 1, 11_000_000)
        assert L.normals % 256 == 0 and L.normals >= L.counters + 16
        assert L.normals + 16 * L.n_flat <= L.total_bytes
        assert L.records == L0.records and L.ranges == L0.ranges and L.counters == L0.counters
        assert L.total_bytes >= L0.total_bytes + 16 * L.n_flat


def test_batch_bases():
    items = (abi.gs_job * 3)()
    for i, (n, W, H) in enumerate([(10, 320, 180), (300, 640, 360), (0, 1920, 1080)]):
        items[i] = fake_job(n, W, H)[0]
    L = R.layout_for(items, 3, 1000)
    assert list(L.gauss_base[:3]) == [0, 256, 256 + 512]
    assert list(L.tile_base[:3]) == [0, 20 * 12, 20 * 12 + 40 * 23]
    assert L.n_tiles == 20 * 12 + 40 * 23 + 120 * 68


def chunk_words(n_flat):
    return -(-n_flat // 256) - (-n_flat // 4096) + 2


def chunk_region_words(L):
    # the chunk-count region ends where the next public region starts
    nxt = min(getattr(L, r) for r in ("tile_keys", "tile_values", "ranges", "counters") if getattr(L, r) > L.chunk_counts)
    return (nxt - L.chunk_counts) // 4


@pytest.mark.parametrize("shapes,bands", [
    ([(960, 540)], 1),                  # 2040 tiles: one pass, no bands
    ([(1920, 1080)], 4),                # 8160 tiles: bands of 17 tile rows (120 x 17 = 2040 tiles)
    ([(2560, 1440)], 8),                # 14400 tiles: bands of 12 rows
    ([(4096, 200)], 2),                 # 256 tiles a row: bands of 8 rows (13 rows)
    ([(640, 360), (320, 180), (512, 1024), (16, 16), (1920, 1080), (97, 61), (960, 540)], 9),
    ([(1280, 720)] * 32, 64),           # two bands per frame: 64 bands, the limit
    ([(1280, 720)] * 33, 1),            # 66 would be needed: the two-pass sort, no bands
])
def test_tile_band_plan(shapes, bands):
    """Over 2048 tiles the chunk counts are kept once per tile band: frames of
    at most 2048 tiles are packed whole in batch order (a new band when the
    next frame would overflow it), larger frames get bands of floor(2048 /
    tiles_x) tile rows of their own, and more than 64 bands fall back to the
    two-pass sort.  The band count shows in the size of the chunk-count
    region (host-only layout call)."""
    items = (abi.gs_job * len(shapes))()
    for i, (W, H) in enumerate(shapes):
        items[i] = fake_job(1000, W, H)[0]
    L = R.layout_for(items, len(shapes), 1_000_000)
    words = chunk_words(L.n_flat)
    assert words * bands <= chunk_region_words(L) < words * bands + 64, (chunk_region_words(L), words)


@pytest.mark.parametrize("mutate", ["n_jobs0", "deg4", "width0", "width_big", "fx0", "near0", "overlap3", "cap_neg",
                                    "too_many"])
def test_invalid_arguments(mutate):
    j = fake_job()
    n_jobs, cap = 1, 1000
    if mutate == "n_jobs0":
        n_jobs = 0
    elif mutate == "deg4":
        j[0].scene.sh_degree = 4
    elif mutate == "width0":
        j[0].cam.width = 0
    elif mutate == "width_big":
        j[0].cam.width = 4097
    elif mutate == "fx0":
        j[0].cam.fx = 0.0
    elif mutate == "near0":
        j[0].opts.near_z = 0.0
    elif mutate == "overlap3":
        j[0].opts.overlap = 3
    elif mutate == "cap_neg":
        cap = -1
    elif mutate == "too_many":
        n_jobs = abi.GS_MAX_BATCH + 1
    L = abi.gs_ws_layout()
    rc = abi.gs_forward_layout(j, n_jobs, cap, 0, C.byref(L))
    assert rc == abi.GS_ERR_INVALID_ARG
    assert abi.last_error()


def test_forward_rejects_small_workspace_without_launching():
    j = fake_job()
    j[0].out.final_T = 256
    j[0].out.n_contrib = 256
    rc = abi.gs_render_forward_batch(j, 1, 256, 1024, 1000, None)
    assert rc == abi.GS_ERR_INVALID_ARG and "workspace" in abi.last_error()


def test_forward_requires_saved_state_outputs():
    j = fake_job()
    rc = abi.gs_render_forward_batch(j, 1, 256, 1 << 40, 1000, None)
    assert rc == abi.GS_ERR_INVALID_ARG and "final_T" in abi.last_error()


@pytest.mark.parametrize("case", ["scale0", "scale5", "width0", "height_big", "null"])
def test_upsample_invalid_arguments(case):
    W, H, S, ptr = 64, 32, 4, 256
    if case == "scale0":
        S = 0
    elif case == "scale5":
        S = 5
    elif case == "width0":
        W = 0
    elif case == "height_big":
        H = 4097
    rgb = None if case == "null" else ptr
    rc = abi.gs_gradient_upsample(rgb, ptr, ptr, W, H, S, ptr, None)
    assert rc == abi.GS_ERR_INVALID_ARG and abi.last_error()


def _cam(width=64, height=32, fx=50.0):
    return R.camera_struct(synth.identity_camera(width, height).replace(fx=fx, fy=fx))


def test_warp_workspace_size():
    n = C.c_size_t(0)
    assert abi.gs_warp_workspace_size(C.byref(_cam(97, 61)), C.byref(_cam(81, 50)), C.byref(n)) == abi.GS_OK
    assert n.value == 97 * 61 * 16 + (81 * 50 + 1) // 2 * 16
    assert abi.gs_warp_workspace_size(C.byref(_cam()), C.byref(_cam(0, 50)), C.byref(n)) == abi.GS_ERR_INVALID_ARG


@pytest.mark.parametrize("case", ["null_alpha", "null_depth", "rgb_missing", "grad_missing", "normal_missing",
                                  "short_ws",
                                  "misaligned_ws", "bad_fx", "big_raster", "nan_pose", "null_out"])
def test_warp_invalid_arguments(case):
    """Rejected before anything is launched (no device needed)."""
    ptr = 1 << 20
    src, dst = _cam(), _cam()
    rgb = alpha = depth = gx = gy = motion = ptr
    out = abi.gs_warp_outputs(ptr, ptr, ptr, ptr, ptr, ptr, ptr)
    nrm = ptr
    ws, ws_bytes = ptr, 64 * 32 * 8 + 64 * 32 * 16
    if case == "null_alpha":
        alpha = None
    elif case == "null_depth":
        depth = None
    elif case == "rgb_missing":
        rgb = None
    elif case == "grad_missing":
        gy = None
    elif case == "normal_missing":
        nrm = None
    elif case == "short_ws":
        ws_bytes -= 8
    elif case == "misaligned_ws":
        ws += 8
    elif case == "bad_fx":
        dst.fx = 0.0
    elif case == "big_raster":
        src.width = 4097
    elif case == "nan_pose":
        dst.t[1] = float("nan")
    rc = abi.gs_motion_warp(C.byref(src), C.byref(dst), rgb, alpha, depth, gx, gy, nrm, motion,
                            None if case == "null_out" else C.byref(out), ws, ws_bytes, None)
    assert rc == abi.GS_ERR_INVALID_ARG and abi.last_error()


@pytest.mark.parametrize("case", ["null", "quats", "sh", "sh_deg2_ok"])
def test_backward_gradient_array_checks(case):
    """Null or misaligned gradient arrays are refused before any launch (a
    degree-2 scene's 27 floats per Gaussian carry no alignment rule)."""
    j = fake_job()
    g = abi.gs_grads(256, 256, 256, 256, 256)
    if case == "null":
        g.opacity_logits = None
    elif case == "quats":
        g.quats = 260
    elif case == "sh":
        g.sh = 264
    else:
        j[0].scene.sh_degree = 2
        g.sh = 260
    rc = abi.gs_render_backward(C.byref(j[0].scene), C.byref(j[0].cam), C.byref(j[0].opts), C.byref(j[0].out),
                                None, 0, 1000, 256, None, None, C.byref(g), None)
    assert rc == abi.GS_ERR_INVALID_ARG
    msg = abi.last_error()
    if case == "sh_deg2_ok":
        assert "aligned" not in msg   # refused later, for the missing forward state
    else:
        assert ("null" if case == "null" else case + " must be 16-byte aligned") in msg


def test_missing_library_fails_loudly(tmp_path, monkeypatch):
    """No fallback: without libgs3.so every entry point raises instead of
    computing anything elsewhere."""
    monkeypatch.setattr(abi, "LIB_PATH", str(tmp_path / "libgs3.so"))
    monkeypatch.setattr(abi, "_lib", None, raising=False)
    with pytest.raises(RuntimeError, match="missing"):
        abi.lib()
    with pytest.raises(RuntimeError, match="missing"):
        abi.gs_gradient_upsample(None, None, None, 1, 1, 1, None, None)
