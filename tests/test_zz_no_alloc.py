"""The forward entry point that allocates nothing (gs_render_forward_noalloc),
through the C ABI, against gs_render_forward_batch on the same frames: two
calls in a row, the second on a smaller frame, outputs and pair counts bit
for bit; a frame beyond the scratch array is refused before any launch."""

import ctypes as C

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2605_11489_amd import abi  # noqa: E402
from paper_2605_11489_amd import render as R  # noqa: E402

KEYS = ("rgb", "alpha", "depth", "dcdx", "dcdy", "final_T", "n_contrib")


def say(msg):
    print(msg, flush=True)


def noalloc(items, key_capacity):
    outs = [it[3] for it in items]
    jobs = R.make_jobs(items)
    counts = torch.full((2,), -1, dtype=torch.int32, device="cuda")
    rc = abi.gs_render_forward_noalloc(jobs, len(items), int(key_capacity), counts.data_ptr(),
                                       R.current_stream_ptr())
    abi.check(rc)
    torch.cuda.synchronize()
    return outs, counts.cpu().numpy()


def reference(items):
    fr = R.render_batch(items)
    rc, k = R.forward_status(fr)
    assert rc == 0
    return fr


def test_noalloc_forward_matches_the_workspace_forward_twice():
    cases = [
        ("1M Gaussians, 960x540", synth.gen_cfg2()[0], synth.cfg2_camera(960, 540), (0.0, 0.0, 0.0)),
        ("3000 Gaussians, 97x61, bg", synth.gen_clustered(81, 3000, 2), synth.look_at_camera((0.7, -0.2, -3.1), 97, 61),
         (0.2, 0.4, 0.6)),
    ]
    for name, scene, cam, bg in cases:
        say(f"case: no-alloc forward, {name}")
        ds = R.DeviceScene.from_host(scene)
        opts = R.opts_struct(bg=bg)
        ref_out = R.alloc_outputs(cam.width, cam.height)
        fr = reference([(ds, cam, opts, ref_out)])
        na_out = R.alloc_outputs(cam.width, cam.height)
        for k in KEYS:
            na_out[k].fill_(7)
        outs, counts = noalloc([(ds, cam, opts, na_out)], fr.key_capacity)
        say(f"  pairs {int(counts[0])} (workspace forward {fr.key_capacity}), overflow flag {int(counts[1])}")
        assert int(counts[0]) == fr.key_capacity and int(counts[1]) == 0
        for k in KEYS:
            assert torch.equal(outs[0][k], ref_out[k]), k


def test_noalloc_forward_batch_and_overflow_flag():
    say("case: no-alloc forward, a batch of two frames, then too small a capacity")
    a, b = synth.gen_clustered(82, 20_000, 3), synth.gen_clustered(83, 8_000, 1)
    ca, cb = synth.look_at_camera((0.3, 0.1, -3.5), 211, 119), synth.look_at_camera((-0.5, 0.4, -2.9), 64, 80)
    da, db = R.DeviceScene.from_host(a), R.DeviceScene.from_host(b)
    ref = [R.alloc_outputs(c.width, c.height) for c in (ca, cb)]
    fr = reference([(da, ca, R.opts_struct(), ref[0]), (db, cb, R.opts_struct(), ref[1])])
    got = [R.alloc_outputs(c.width, c.height) for c in (ca, cb)]
    outs, counts = noalloc([(da, ca, R.opts_struct(), got[0]), (db, cb, R.opts_struct(), got[1])], fr.key_capacity)
    assert int(counts[0]) == fr.key_capacity and int(counts[1]) == 0
    for j in range(2):
        for k in KEYS:
            assert torch.equal(outs[j][k], ref[j][k]), (j, k)
    _, counts = noalloc([(da, ca, R.opts_struct(), got[0])], 100)
    assert int(counts[1]) != 0 and int(counts[0]) > 100


def test_noalloc_forward_refuses_a_frame_beyond_the_scratch():
    say("case: no-alloc forward, 6M Gaussians at 1920x1080 (needs ~6 GB) is refused")
    j = (abi.gs_job * 1)()
    j[0].scene = abi.gs_scene(256, 256, 256, 256, 256, 6_000_000, 3, 0)
    j[0].cam = R.camera_struct(synth.cfg2_camera(1920, 1080))
    j[0].opts = R.opts_struct()
    j[0].out = abi.gs_outputs(None, None, None, None, None, 256, 256, None, None, None, None)
    rc = abi.gs_render_forward_noalloc(j, 1, 186_000_000, None, None)
    assert rc == abi.GS_ERR_TOO_LARGE
    assert "scratch" in abi.last_error()
