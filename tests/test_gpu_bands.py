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
from tests.parity import compare_frame, gpu_outputs_numpy  # noqa: E402


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


def hot_tile_scene(seed, n_hot, n_background, W, H, tile):
    """n_hot Gaussians of about 2 pixels' footprint whose every pixel lies in
    one 16x16 tile (identity camera, depths 3..5), and a background spread
    over the frame."""
    rng = np.random.default_rng(seed)
    cam = synth.identity_camera(W, H)
    tx, ty = tile
    u = rng.uniform(16 * tx + 4, 16 * tx + 12, n_hot)
    v = rng.uniform(16 * ty + 4, 16 * ty + 12, n_hot)
    z = rng.uniform(3.0, 5.0, n_hot)
    means = np.stack([(u - cam.cx) * z / cam.fx, (v - cam.cy) * z / cam.fy, z], axis=1)
    bg = synth.random_scene_small(seed + 1, n_background, 0, log_scale_mean=-6.0)
    quats = rng.normal(size=(n_hot, 4))
    sh = np.zeros((n_hot, 1, 3), np.float32)
    sh[:, 0, :] = rng.uniform(-1.0, 1.0, (n_hot, 3))
    hot = synth.Scene(means.astype(np.float32), np.full((n_hot, 3), np.log(6e-4), np.float32),
                      (quats / np.linalg.norm(quats, axis=1, keepdims=True)).astype(np.float32),
                      rng.normal(0.0, 1.0, n_hot).astype(np.float32), sh, 0)
    scene = synth.Scene(*(np.concatenate([getattr(hot, f), getattr(bg, f)]) for f in
                          ("means", "log_scales", "quats", "opacity_logits", "sh")), 0)
    return scene, cam


@pytest.mark.parametrize("W,H,tile", [(1920, 1080, (60, 30)), (960, 540, (30, 20))])
def test_long_run_of_one_tile_in_a_band(W, H, tile):
    """100k pairs of one tile, nearly all of its band's pairs (1920x1080,
    banded: blocks of 8192 in groups of 8) or of the frame's (960x540, one
    pass: blocks of 4096 in groups of 16): a block's 16-bit count prefix
    inside its histogram group reaches 7 x 8192 or 15 x 4096 and no further
    (a group of 16 blocks of 8192 would pass 65535).  Keys, values and
    ranges equal the oracle's, and so does the hot tile's compositing."""
    scene, cam = hot_tile_scene(47, 100_000, 3000, W, H, tile)
    of = oracle.render_forward(scene, cam, composite_all=False)
    lens = of.ranges[:, 1] - of.ranges[:, 0]
    t = tile[1] * ((W + 15) // 16) + tile[0]
    say(f"case: {W}x{H}, {scene.n} Gaussians, {lens[t]} pairs on tile {tile} of {of.keys.size}")
    assert lens[t] >= 100_000
    fr, _ = render_items([(scene, cam)])
    rc, k = R.forward_status(fr)
    assert rc == 0 and k == of.keys.size
    check_frame(fr, 0, of)
    tiles = [t, t + 1]
    of.image = oracle.composite.composite_image(of.proj, of.values, of.ranges, W, H, of.bg, tiles=tiles)
    st = compare_frame(gpu_outputs_numpy(fr.outputs[0]), of, tiles=tiles)
    say(f"  pixels={st['pixels']} clean_max_err={st['clean_max_err']:.3g} flipped={st['flipped']}")
    assert not st["unresolved"], st["unresolved"][:5]
    assert st["clean_max_err"] <= 1e-4


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
