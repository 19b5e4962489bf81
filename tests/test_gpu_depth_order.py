"""The depth sort on the GPU against its definition: the 2D Gaussians in the
order of their 32-bit view-z keys (Sec. 3: the Gaussians are depth-sorted),
equal keys in index order, culled Gaussians (key 0xFFFFFFFF) last, and each
packed tile rectangle carried to its Gaussian's sorted position.  The keys
are the GPU's own (the projection tests check them against the oracle bit
for bit); the reference order is a stable argsort of them.  Cases cover the
small-pass path (fewer than 4M keys, 1024-thread blocks) with ragged counts,
heavily duplicated keys and culled Gaussians between visible ones, and the
large-pass path (512-thread blocks) over 4.2M keys."""

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2605_11489_amd import render as R  # noqa: E402

CULLED = 0xFFFFFFFF


def say(msg):
    print(msg, flush=True)


def check_depth_sort(scene, cam):
    ds = R.DeviceScene.from_host(scene)
    fr = R.render(ds, cam)
    rc, _ = R.forward_status(fr)
    assert rc == 0
    L, ws = fr.layout, fr.workspace
    n = int(L.n_flat)

    def words(off):
        return ws[off:off + 4 * n].cpu().numpy().view(np.uint32)

    key, rect, order, drect = words(L.depth_keys), words(L.rects), words(L.depth_order), words(L.depth_rects)
    culled = int(np.count_nonzero(key == CULLED))
    distinct = np.unique(key[key != CULLED]).size
    say(f"  {n} flat Gaussians, {culled} culled, {distinct} distinct live keys")
    ref = np.lexsort((np.arange(n), key))   # by key, then index
    assert np.array_equal(order, ref.astype(np.uint32)), "depth order differs from the stable argsort"
    assert np.array_equal(drect, rect[ref]), "rectangles not carried to their sorted positions"
    return culled, distinct, n


def test_depth_order_config1():
    say("case: 10k Gaussians, 256x256 (three small passes)")
    check_depth_sort(*synth.gen_cfg1())


def test_depth_order_duplicates_and_culled_between():
    """12289 Gaussians (three blocks of 4096 and one more): their depths
    snapped to 8 values, so most keys repeat thousands of times, and every
    third Gaussian behind the camera (culled) between visible ones."""
    say("case: 12289 Gaussians, 8 distinct depths, a third behind the camera")
    scene = synth.random_scene_small(61, 12289, 0, log_scale_mean=-4.0)
    rng = np.random.default_rng(62)
    z = rng.choice(np.array([2.0, 2.5, 3.0, 3.25, 4.0, 4.5, 5.0, 6.0], np.float32), scene.n)
    z[::3] = -3.0
    scene.means[:, 2] = z
    culled, distinct, _ = check_depth_sort(scene, synth.identity_camera(640, 360))
    assert culled >= 12289 // 3 and distinct <= 8


def test_depth_order_large_pass():
    """4.2M Gaussians (the passes over 4M keys or more: two launches to fold
    the block histograms, 512-thread scatters)."""
    say("case: 4.2M Gaussians, 960x540")
    scene = synth.gen_clustered(63, 4_200_000, 0)
    _, _, n = check_depth_sort(scene, synth.cfg2_camera())
    assert n >= 4 << 20
