"""The banded tile sort (batches over 2048 tiles) against the FP64 oracle.

Over 2048 tiles the pairs are emitted into tile bands of at most 2048 tiles:
frames packed whole into a band, or the row bands of one large frame.  Each
band is sorted by one radix pass on band-local tile ids.  These tests check,
per frame, that the sorted keys, values and tile ranges are bit-identical to
the oracle's, across the packing rules (whole frames sharing a band, a frame
of exactly 2048 tiles, 4096-pixel-wide frames of 8-row bands, bands without
any pair), the capacity overflow path, and the fallback to two passes when a
batch would need more than 64 bands."""

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2605_11489_amd import abi, render as R  # noqa: E402


def say(msg):
    print(msg, flush=True)


def tiles_of(cam):
    return ((cam.width + 15) // 16) * ((cam.height + 15) // 16)


def frame_ranges(fr, j, nt):
    L = fr.layout
    t0 = int(L.tile_base[j])
    raw = fr.workspace[L.ranges + 8 * t0:L.ranges + 8 * (t0 + nt)].cpu().numpy()
    return raw.view(np.uint32).reshape(nt, 2).astype(np.int64)


def check_frame(fr, j, of):
    """Keys, values and ranges of job j of a batch equal the oracle's frame;
    the ranges are the oracle's shifted by the pairs of the tiles before the
    frame (empty tiles are [0, 0] in both)."""
    keys, vals = R.sorted_keys(fr, j, count=int(of.keys.size))
    assert np.array_equal(keys, of.keys), f"job {j}: sorted keys differ"
    assert np.array_equal(vals, of.values), f"job {j}: sorted values differ"
    nt = of.ranges.shape[0]
    rg = frame_ranges(fr, j, nt)
    full = of.ranges[:, 1] > of.ranges[:, 0]
    assert np.array_equal(rg[~full], of.ranges[~full]), f"job {j}: empty tile ranges differ"
    if full.any():
        shift = rg[full][0, 0] - of.ranges[full][0, 0]
        assert np.array_equal(rg[full] - shift, of.ranges[full]), f"job {j}: tile ranges differ"


def render_items(items, key_capacity=None):
    devs = []
    batch = []
    for scene, cam in items:
        ds = R.DeviceScene.from_host(scene)
        devs.append(ds)
        batch.append((ds, cam, R.opts_struct(), R.alloc_outputs(cam.width, cam.height)))
    fr = R.render_batch(batch, key_capacity=key_capacity)
    return fr, devs


def test_mixed_batch_packs_and_splits_bands():
    """Small frames packed into shared bands, a frame of exactly 2048 tiles
    alone in its band, a 1080p frame cut into four row bands, and a 16x16
    frame after it: every frame's keys, values and ranges equal the oracle's,
    and its image equals the same frame rendered alone."""
    shapes = [(640, 360), (320, 180), (512, 1024), (16, 16), (1920, 1080), (97, 61), (960, 540)]
    items = []
    for k, (W, H) in enumerate(shapes):
        scene = synth.gen_clustered(300 + k, 4000 + 500 * k, k % 4)
        items.append((scene, synth.look_at_camera((0.5 - 0.1 * k, -0.3, -3.2), W, H)))
    say("case: mixed batch " + ", ".join(f"{W}x{H}" for W, H in shapes) +
        f" ({sum(tiles_of(c) for _, c in items)} tiles)")
    fr, devs = render_items(items)
    rc, k = R.forward_status(fr)
    assert rc == 0, (rc, k)
    for j, (scene, cam) in enumerate(items):
        of = oracle.render_forward(scene, cam, composite_all=False)
        check_frame(fr, j, of)
        alone = R.render(devs[j], cam)
        assert R.forward_status(alone)[0] == 0
        for key in ("rgb", "alpha", "depth", "dcdx", "dcdy", "final_T", "n_contrib"):
            assert torch.equal(fr.outputs[j][key], alone.outputs[0][key]), (j, key)
        say(f"  job {j} {cam.width}x{cam.height}: {of.keys.size} pairs identical")


@pytest.mark.parametrize("W,H,ylo,yhi", [(1920, 1080, -0.62, -0.45), (4096, 200, -0.05, -0.02)])
def test_bands_without_pairs(W, H, ylo, yhi):
    """Gaussians only in the upper part of the frame: the lower bands hold
    no pair, yet their tiles' ranges are written ([0, 0]) and the keys stay
    exact.  4096 pixels wide is 256 tiles a row, so a band is 8 tile rows."""
    say(f"case: {W}x{H}, Gaussians in the top rows only")
    scene = synth.random_scene_small(41, 3000, 1, lo=(-1.0, ylo, 2.0), hi=(1.0, yhi, 6.0), log_scale_mean=-6.0)
    cam = synth.identity_camera(W, H)
    fr, _ = render_items([(scene, cam)])
    rc, k = R.forward_status(fr)
    assert rc == 0
    of = oracle.render_forward(scene, cam, composite_all=False)
    lens = of.ranges[:, 1] - of.ranges[:, 0]
    tx = (W + 15) // 16
    rows_with_pairs = np.nonzero(lens.reshape(-1, tx).sum(axis=1))[0]
    say(f"  pairs={of.keys.size} tile rows with pairs {rows_with_pairs.min()}..{rows_with_pairs.max()}"
        f" of {lens.size // tx}")
    rows_per_band = 2048 // tx
    n_bands = -(-(lens.size // tx) // rows_per_band)
    assert rows_with_pairs.max() // rows_per_band < n_bands - 1, "the last band must hold no pair"
    check_frame(fr, 0, of)


def test_banded_capacity_overflow_then_exact():
    """A 1080p frame rendered with fewer key slots than pairs reports the
    capacity error and the pair count (the emission and the banded sort stay
    inside the capacity); at exactly the pair count it is exact."""
    scene = synth.gen_clustered(44, 30_000, 2)
    cam = synth.look_at_camera((0.4, -0.3, -3.0), 1920, 1080)
    of = oracle.render_forward(scene, cam, composite_all=False)
    need = int(of.keys.size)
    say(f"case: 1920x1080 banded, {need} pairs, capacity {need // 2} then {need}")
    fr, devs = render_items([(scene, cam)], key_capacity=need // 2)
    rc, k = R.forward_status(fr)
    assert rc == abi.GS_ERR_CAPACITY and k == need, (rc, k)
    fr2 = R.render_batch([(devs[0], cam, R.opts_struct(), R.alloc_outputs(1920, 1080))], key_capacity=need)
    rc, k = R.forward_status(fr2)
    assert rc == 0 and k == need
    check_frame(fr2, 0, of)


@pytest.mark.parametrize("frames,expect_banded", [(32, True), (33, False)])
def test_band_limit_and_two_pass_fallback(frames, expect_banded):
    """1280x720 frames take two bands each: 32 of them fill the 64 bands,
    33 would need 66 and take the two-pass sort instead.  Both give every
    frame's exact keys and ranges."""
    say(f"case: {frames} frames of 1280x720 ({'banded' if expect_banded else 'two passes'})")
    items = []
    for k in range(frames):
        scene = synth.random_scene_small(500 + k, 400, 0)
        items.append((scene, synth.identity_camera(1280, 720)))
    fr, _ = render_items(items)
    rc, _ = R.forward_status(fr)
    assert rc == 0
    for j in (0, frames // 2, frames - 1):
        scene, cam = items[j]
        of = oracle.render_forward(scene, cam, composite_all=False)
        check_frame(fr, j, of)
    say("  jobs 0, middle and last identical")
