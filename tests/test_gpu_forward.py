"""Forward-pass parity of the HIP path (through the C ABI) against the FP64
oracle: projection records and tile rectangles, sorted keys / values and
tile ranges bit for bit, images and image gradients within 1e-4."""

import numpy as np
import pytest

import oracle
import synth
from oracle import parallel
from tests.parity import compare_frame, gpu_outputs_numpy

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2605_11489_amd import render as R  # noqa: E402


def say(msg):
    print(msg, flush=True)


def run_case(scene, cam, bg=(0.0, 0.0, 0.0)):
    ds = R.DeviceScene.from_host(scene)
    fr = R.render(ds, cam, bg=bg)
    rc, k = R.forward_status(fr)
    assert rc == 0, (rc, k)
    return ds, fr


def record_arrays(fr, n):
    L = fr.layout
    ws = fr.workspace
    raw = ws[L.records:L.records + 48 * n].cpu().numpy()
    f64 = raw.view(np.float64).reshape(n, 6)
    f32 = raw.view(np.float32).reshape(n, 12)
    zkey = ws[L.depth_keys:L.depth_keys + 4 * n].cpu().numpy().view(np.uint32)
    rect = ws[L.rects:L.rects + 4 * n].cpu().numpy().view(np.uint8).reshape(n, 4).astype(np.int64)
    touched = ws[L.touched:L.touched + 4 * n].cpu().numpy().view(np.uint32).astype(np.int64)
    return dict(u=f64[:, 0], v=f64[:, 1], conic=f32[:, 4:7], o=f32[:, 7], rgb=f32[:, 8:11], z=f32[:, 11],
                zkey=zkey, rect=rect, touched=touched)


def check_projection(fr, of):
    P = of.proj
    n = P.n
    g = record_arrays(fr, n)
    vis = P.touched > 0
    assert np.array_equal(g["touched"], P.touched), "tile counts differ"
    assert np.array_equal(g["rect"][vis], P.rect[vis])
    assert np.array_equal(g["zkey"][vis], P.zkey[vis])
    # the 2D mean is formed by the same IEEE operations in the same order
    assert np.array_equal(g["u"][vis], P.u[vis])
    assert np.array_equal(g["v"][vis], P.v[vis])
    assert np.allclose(g["conic"][vis], P.conic[vis], rtol=2e-6, atol=0)
    assert np.abs(g["o"][vis] - P.opacity[vis]).max(initial=0) < 2e-7
    assert np.abs(g["rgb"][vis] - P.rgb[vis]).max(initial=0) < 2e-6


def check_keys(fr, of):
    keys, vals = R.sorted_keys(fr, 0, count=int(of.keys.size))
    assert np.array_equal(keys, of.keys), "sorted keys differ"
    assert np.array_equal(vals, of.values), "sorted values differ"
    L = fr.layout
    nt = of.ranges.shape[0]
    rg = fr.workspace[L.ranges:L.ranges + 8 * nt].cpu().numpy().view(np.uint32).reshape(nt, 2).astype(np.int64)
    assert np.array_equal(rg, of.ranges), "tile ranges differ"


def check_image(fr, of, tiles=None):
    g = gpu_outputs_numpy(fr.outputs[0])
    st = compare_frame(g, of, tiles=tiles)
    say(f"  pixels={st['pixels']} clean_max_err={st['clean_max_err']:.3g} flipped={st['flipped']} "
        f"unresolved={len(st['unresolved'])}")
    assert not st["unresolved"], st["unresolved"][:5]
    assert st["clean_max_err"] <= 1e-4
    return st


def test_config1_full_frame():
    say("case: 10k Gaussians, 256x256, SH deg 0, seed 0")
    scene, cam = synth.gen_cfg1()
    ds, fr = run_case(scene, cam)
    of = oracle.render_forward(scene, cam)
    check_projection(fr, of)
    check_keys(fr, of)
    check_image(fr, of)


@pytest.mark.parametrize("seed,W,H,deg", [(21, 100, 70, 3), (22, 33, 17, 1), (23, 16, 16, 2), (24, 1, 1, 3)])
def test_ragged_rotated_camera(seed, W, H, deg):
    say(f"case: ragged seed={seed} {W}x{H} deg={deg}")
    scene = synth.gen_clustered(seed, 3000, deg)
    cam = synth.look_at_camera((1.2, -0.7, -3.6), W, H)
    bg = (0.25, 0.5, 0.75)
    ds, fr = run_case(scene, cam, bg)
    of = oracle.render_forward(scene, cam, bg=bg)
    check_projection(fr, of)
    check_keys(fr, of)
    check_image(fr, of)


def test_nothing_visible():
    say("case: every Gaussian behind the camera")
    scene = synth.random_scene_small(30, 200, 0, lo=(-1, -1, -5), hi=(1, 1, -1))
    cam = synth.identity_camera(40, 24)
    ds, fr = run_case(scene, cam, bg=(0.1, 0.2, 0.3))
    g = gpu_outputs_numpy(fr.outputs[0])
    assert np.allclose(g["rgb"], np.array([0.1, 0.2, 0.3])[:, None, None])
    assert np.all(g["alpha"] == 0) and np.all(g["n_contrib"] == 0) and np.all(g["final_T"] == 1)
    assert np.all(g["dcdx"] == 0) and np.all(g["depth"] == 0)


def test_config2_full_size_keys_and_full_frame_image():
    """The benchmark's frame (1M Gaussians, 960x540) in full: projection and
    keys bit for bit, and every one of the 2040 tiles' images and gradient
    buffers against the oracle (composited over worker processes)."""
    say("case: 1M Gaussians in 64 clusters, 960x540, SH deg 3, seed 0, all 2040 tiles")
    scene, cam = synth.gen_cfg2()
    ds, fr = run_case(scene, cam)
    of = oracle.render_forward(scene, cam, composite_all=False)
    say(f"  keys={of.keys.size}")
    check_projection(fr, of)
    check_keys(fr, of)
    tm = {}
    of.image = parallel.composite_image_parallel(of.proj, of.values, of.ranges, 960, 540, of.bg, timing=tm)
    iy, ix = np.mgrid[0:540, 0:960]
    of.image.nv = oracle.composite.normal_view(of.image.normal, cam, ix, iy)
    say(f"  oracle composited {len(of.image.tiles)} tiles in {tm['composite_s']:.1f} s on {tm['workers']} processes")
    st = check_image(fr, of)
    assert st["pixels"] == 960 * 540


@pytest.mark.parametrize("cfg", ["c1", "ragged"])
def test_wide_list_positions(cfg):
    """With a key capacity of 2^28 or more the compositing kernel keeps the
    last blended list position as a plain index (the kWide variants); its
    outputs, n_contrib included, equal the narrow variant's bit for bit and
    the oracle's within 1e-4, and the backward over that frame gives the
    narrow frame's gradients."""
    say(f"case: wide compositing variant (key capacity 2^28), {cfg}")
    if cfg == "c1":
        scene, cam = synth.gen_cfg1()
        bg = (0.0, 0.0, 0.0)
    else:
        scene = synth.gen_clustered(25, 4000, 2)
        cam = synth.look_at_camera((1.1, -0.6, -3.3), 101, 67)
        bg = (0.3, 0.5, 0.7)
    ds = R.DeviceScene.from_host(scene)
    opts = R.opts_struct(bg=bg)
    out_w = R.alloc_outputs(cam.width, cam.height)
    fr_w = R.render_batch([(ds, cam, opts, out_w)], key_capacity=1 << 28, with_backward=True)
    assert R.forward_status(fr_w)[0] == 0
    out_n = R.alloc_outputs(cam.width, cam.height)
    fr_n = R.render_batch([(ds, cam, opts, out_n)], with_backward=True)
    assert R.forward_status(fr_n)[0] == 0
    assert fr_n.key_capacity < (1 << 28)
    for k in ("rgb", "alpha", "depth", "dcdx", "dcdy", "final_T", "n_contrib"):
        assert torch.equal(out_w[k], out_n[k]), k
    of = oracle.render_forward(scene, cam, bg=bg)
    check_keys(fr_w, of)
    check_image(fr_w, of)
    # the backward reads n_contrib as a list position: the wide frame's gradients
    rng = np.random.default_rng(26)
    g_rgb = torch.from_numpy(rng.normal(size=(3, cam.height, cam.width)).astype(np.float32)).cuda()
    grads = {}
    for name, fr, out in (("wide", fr_w, out_w), ("narrow", fr_n, out_n)):
        gl = [torch.zeros_like(t) for t in ds.tensors()]
        R.render_backward(fr, g_rgb, gl)
        grads[name] = [g.cpu().numpy().astype(np.float64) for g in gl]
    from oracle import backward as OB
    g2 = OB.composite_backward(of, g_rgb.cpu().numpy().astype(np.float64))
    pg = OB.project_backward(scene, cam, of.proj, g2)
    for i, f in enumerate(("means", "log_scales", "quats", "opacity_logits", "sh")):
        ref = getattr(pg, f)
        scale = max(1.0, float(np.abs(ref).max()))
        assert np.abs(grads["wide"][i] - grads["narrow"][i]).max() <= 1e-5 * scale, f
        assert np.abs(grads["wide"][i] - ref).max() <= 1e-4 * scale, f


@pytest.mark.parametrize("W,H", [(1280, 720), (1920, 1080), (2560, 1440)])
def test_large_rasters(W, H):
    """Over 2048 tiles (3600, 8160 and 14400 here: 2, 4 and 8 bands of tile
    rows) the pairs are emitted per tile band and each band is sorted by one
    pass on band-local tile ids; keys and ranges stay bit-exact."""
    say(f"case: 60k Gaussians, {W}x{H} ({((W + 15) // 16) * ((H + 15) // 16)} tiles), seed 71")
    scene = synth.gen_clustered(71, 60_000, 3)
    cam = synth.look_at_camera((0.6, -0.4, -3.5), W, H)
    ds, fr = run_case(scene, cam)
    of = oracle.render_forward(scene, cam, composite_all=False)
    say(f"  keys={of.keys.size}")
    check_projection(fr, of)
    check_keys(fr, of)
    rng = np.random.default_rng(7)
    nt = of.ranges.shape[0]
    lens = of.ranges[:, 1] - of.ranges[:, 0]
    tiles = sorted(set(rng.choice(nt, 6, replace=False).tolist()) | {int(np.argmax(lens)), nt - 1})
    of.image = oracle.composite.composite_image(of.proj, of.values, of.ranges, W, H, of.bg, tiles=tiles)
    check_image(fr, of, tiles)


def test_pair_counters_match_oracle():
    say("case: per-pixel evaluated / blended pair counts, 10k Gaussians 256x256")
    scene, cam = synth.gen_cfg1()
    ds = R.DeviceScene.from_host(scene)
    out = R.alloc_outputs(cam.width, cam.height)
    out["n_evaluated"] = torch.empty(cam.height, cam.width, dtype=torch.int32, device="cuda")
    out["n_blended"] = torch.empty(cam.height, cam.width, dtype=torch.int32, device="cuda")
    fr = R.render_batch([(ds, cam, R.opts_struct(), out)])
    assert R.forward_status(fr)[0] == 0
    of = oracle.render_forward(scene, cam)
    ev = out["n_evaluated"].cpu().numpy()
    bl = out["n_blended"].cpu().numpy()
    amb = np.zeros(ev.shape, dtype=bool)
    for (ix, iy) in of.image.ambiguous:
        amb[iy, ix] = True
    assert np.array_equal(ev[~amb], of.image.evaluated[~amb])
    assert np.array_equal(bl[~amb], of.image.blended[~amb])
    # the counting variant renders the same image as the plain kernel
    fr2 = R.render(ds, cam)
    assert R.forward_status(fr2)[0] == 0
    for k in ("rgb", "dcdx", "final_T", "n_contrib"):
        assert torch.equal(out[k], fr2.outputs[0][k])


@pytest.mark.parametrize("cfg", ["c2", "ragged"])
def test_quadrant_culling_is_exact(cfg):
    """The compositing kernel skips (Gaussian, 8x8 quadrant) pairs that cannot
    reach alpha >= 1/255; its counting variant walks every pair.  Both must
    render identical bits."""
    say(f"case: quadrant culling vs full walk, {cfg}")
    if cfg == "c2":
        scene, cam = synth.gen_cfg2()
    else:
        scene = synth.gen_clustered(61, 20_000, 2)
        cam = synth.look_at_camera((0.9, 0.3, -2.2), 203, 117)
    ds = R.DeviceScene.from_host(scene)
    out = R.alloc_outputs(cam.width, cam.height)
    out["n_evaluated"] = torch.empty(cam.height, cam.width, dtype=torch.int32, device="cuda")
    fr = R.render_batch([(ds, cam, R.opts_struct(bg=(0.3, 0.6, 0.9)), out)])
    assert R.forward_status(fr)[0] == 0
    fr2 = R.render(ds, cam, bg=(0.3, 0.6, 0.9))
    assert R.forward_status(fr2)[0] == 0
    for k in ("rgb", "alpha", "depth", "dcdx", "dcdy", "final_T", "n_contrib"):
        assert torch.equal(out[k], fr2.outputs[0][k]), k


def _pairs(keys, vals):
    return (keys >> np.uint64(32)).astype(np.int64) * (1 << 32) + vals.astype(np.int64)


@pytest.mark.parametrize("mode", [1, 2])
@pytest.mark.parametrize("cfg", ["c2", "c2_1080p", "ragged"])
def test_opacity_overlap_is_exact(cfg, mode):
    """Opacity-aware tile overlap (mode 1: the ellipse's bounding box; mode
    2: the tiles the ellipse reaches, row by row) drops only pairs whose alpha
    stays below 1/255 over the whole tile: every image buffer is
    bit-identical to the 3-sigma square's, and its pairs are a subset of the
    square's (mode 2's also of mode 1's)."""
    say(f"case: overlap mode {mode} vs 3-sigma square, {cfg}")
    if cfg == "c2":
        scene, cam = synth.gen_cfg2()
    elif cfg == "c2_1080p":
        # 8160 tiles: the square and box modes take the banded tile sort, the
        # ellipse mode two passes and a boundary scan
        scene, _ = synth.gen_cfg2()
        cam = synth.cfg2_camera(1920, 1080)
    else:
        scene = synth.gen_clustered(62, 20_000, 2)
        cam = synth.look_at_camera((0.7, -0.5, -2.4), 203, 117)
    bg = (0.3, 0.6, 0.9)
    ds = R.DeviceScene.from_host(scene)
    frames = {}
    for m in sorted({0, 1, mode}):
        out = R.alloc_outputs(cam.width, cam.height)
        fr = R.render_batch([(ds, cam, R.opts_struct(bg=bg, overlap=m), out)])
        rc, k = R.forward_status(fr)
        assert rc == 0
        frames[m] = (fr, out, k)
    for key in ("rgb", "alpha", "depth", "dcdx", "dcdy", "final_T"):
        assert torch.equal(frames[0][1][key], frames[mode][1][key]), key
    k0, k1 = frames[0][2], frames[mode][2]
    say(f"  pairs square={k0} mode {mode}={k1} ({k1 / max(k0, 1):.3f})")
    assert k1 <= k0 and k1 <= frames[1][2]
    ks, vs = R.sorted_keys(frames[0][0], 0, count=k0)
    kt, vt = R.sorted_keys(frames[mode][0], 0, count=k1)
    ps, pt = _pairs(ks, vs), _pairs(kt, vt)
    assert np.all(np.isin(pt, ps)), "the pairs must be a subset of the square's"
    # within each tile the list keeps the square's order (sorted keys, ties by index)
    assert np.all(kt[1:] >= kt[:-1])
    if mode == 2:
        k1b, v1b = R.sorted_keys(frames[1][0], 0, count=frames[1][2])
        assert np.all(np.isin(pt, _pairs(k1b, v1b))), "ellipse pairs must be a subset of the bounding box's"
    if cfg == "ragged":
        # every dropped pair: alpha' < 1/255 at all pixel centres of its tile (FP64 oracle)
        of = oracle.render_forward(scene, cam, composite_all=False)
        P = of.proj
        dropped = np.setdiff1d(ps, pt)
        tiles = dropped >> 32
        gs = dropped & 0xFFFFFFFF
        tx_n = (cam.width + 15) // 16
        amin = float(np.float32(1 / 255))
        worst = 0.0
        for t, g in zip(tiles.tolist(), gs.tolist()):
            x0, y0 = (t % tx_n) * 16, (t // tx_n) * 16
            px = np.arange(x0, min(x0 + 16, cam.width)) + 0.5
            py = np.arange(y0, min(y0 + 16, cam.height)) + 0.5
            X, Y = np.meshgrid(px, py)
            dx, dy = P.u[g] - X, P.v[g] - Y
            A, B, C = P.conic[g]
            a = P.opacity[g] * np.exp(-0.5 * (A * dx * dx + 2 * B * dx * dy + C * dy * dy))
            worst = max(worst, float(a.max()))
        say(f"  dropped={dropped.size} max alpha' over their tiles={worst:.3g}")
        assert dropped.size > 0 and worst < amin


def test_ellipse_overlap_in_a_mixed_batch():
    """A batch mixing the ellipse mode with the square and box modes (one
    emission launch takes both paths): every frame's outputs and sorted
    pairs equal those of the same frame rendered alone."""
    say("case: batch of overlap modes 2, 0, 1 against single renders")
    items = []
    for k, (seed, n, deg, eye, W, H, mode) in enumerate([(62, 20_000, 2, (0.7, -0.5, -2.4), 203, 117, 2),
                                                         (63, 5_000, 3, (0.2, 0.3, -3.0), 96, 80, 0),
                                                         (64, 8_000, 1, (-0.5, 0.1, -2.8), 130, 47, 1)]):
        scene = synth.gen_clustered(seed, n, deg)
        cam = synth.look_at_camera(eye, W, H)
        items.append((R.DeviceScene.from_host(scene), cam, mode))
    outs = [R.alloc_outputs(c.width, c.height) for _, c, _ in items]
    frb = R.render_batch([(ds, c, R.opts_struct(overlap=m), o) for (ds, c, m), o in zip(items, outs)])
    rc, _ = R.forward_status(frb)
    assert rc == 0
    for j, ((ds, cam, mode), ob) in enumerate(zip(items, outs)):
        o1 = R.alloc_outputs(cam.width, cam.height)
        fr1 = R.render_batch([(ds, cam, R.opts_struct(overlap=mode), o1)])
        rc, k1 = R.forward_status(fr1)
        assert rc == 0
        for key in ("rgb", "alpha", "depth", "dcdx", "dcdy", "final_T", "n_contrib"):
            assert torch.equal(ob[key], o1[key]), (j, key)
        kb, vb = R.sorted_keys(frb, j)
        ks, vs = R.sorted_keys(fr1, 0, count=k1)
        assert np.array_equal(kb, ks) and np.array_equal(vb, vs), j
        say(f"  frame {j} (mode {mode}): {k1} pairs, identical")


def test_ellipse_overlap_large_gaussians():
    """Gaussians spanning ~30 tile rows at 1920x1080, so a block's box rows
    overflow the emission's LDS row table and most Gaussians take the row
    walk instead: images still bit-identical to the square mode, pairs a
    subset of the square's."""
    say("case: ellipse overlap, large Gaussians at 1920x1080 (row-table overflow path)")
    scene = synth.random_scene_small(71, 2000, 1, log_scale_mean=-1.5, log_scale_std=0.3)
    cam = synth.identity_camera(1920, 1080)
    ds = R.DeviceScene.from_host(scene)
    frames = {}
    for m in (0, 2):
        out = R.alloc_outputs(cam.width, cam.height)
        fr = R.render_batch([(ds, cam, R.opts_struct(bg=(0.1, 0.2, 0.3), overlap=m), out)])
        rc, k = R.forward_status(fr)
        assert rc == 0
        frames[m] = (fr, out, k)
    for key in ("rgb", "alpha", "depth", "dcdx", "dcdy", "final_T"):
        assert torch.equal(frames[0][1][key], frames[2][1][key]), key
    k0, k2 = frames[0][2], frames[2][2]
    say(f"  pairs square={k0} ellipse={k2}")
    assert k2 < k0
    ks, vs = R.sorted_keys(frames[0][0], 0, count=k0)
    kt, vt = R.sorted_keys(frames[2][0], 0, count=k2)
    assert np.all(np.isin(_pairs(kt, vt), _pairs(ks, vs)))


@pytest.mark.parametrize("mode", [1, 2])
def test_overlap_modes_keep_normal_maps(mode):
    """The normal and normal-view maps (f2) are blended over the same pairs,
    so the box and ellipse overlaps leave them bit-identical too."""
    say(f"case: normal maps under overlap mode {mode}")
    scene = synth.gen_clustered(65, 30_000, 3)
    cam = synth.look_at_camera((0.4, -0.3, -2.6), 211, 119)
    ds = R.DeviceScene.from_host(scene)
    outs = {}
    for m in (0, mode):
        out = R.alloc_outputs(cam.width, cam.height, normals=True)
        fr = R.render_batch([(ds, cam, R.opts_struct(bg=(0.2, 0.2, 0.2), overlap=m), out)])
        rc, _ = R.forward_status(fr)
        assert rc == 0
        outs[m] = out
    for key in ("rgb", "alpha", "depth", "dcdx", "dcdy", "final_T", "normal", "nv"):
        assert torch.equal(outs[0][key], outs[mode][key]), key


def test_batch_of_large_frames():
    """Two 1920x1080 frames in one batch (16320 global tiles in 8 bands; both
    frames' Gaussians interleaved in depth order): each frame's keys, ranges
    and images equal the same frame rendered alone."""
    say("case: batch of two 1920x1080 frames vs single renders")
    a, b = synth.gen_clustered(72, 40_000, 2), synth.gen_clustered(73, 30_000, 1)
    ca, cb = synth.look_at_camera((0.6, -0.4, -3.5), 1920, 1080), synth.look_at_camera((-0.4, 0.2, -3.0), 1920, 1080)
    da, db = R.DeviceScene.from_host(a), R.DeviceScene.from_host(b)
    outs = [R.alloc_outputs(1920, 1080) for _ in range(2)]
    frb = R.render_batch([(da, ca, R.opts_struct(), outs[0]), (db, cb, R.opts_struct(), outs[1])])
    assert R.forward_status(frb)[0] == 0
    for j, (ds, cam) in enumerate(((da, ca), (db, cb))):
        fr1 = R.render(ds, cam)
        rc, k1 = R.forward_status(fr1)
        assert rc == 0
        for key in ("rgb", "alpha", "depth", "dcdx", "dcdy", "final_T", "n_contrib"):
            assert torch.equal(outs[j][key], fr1.outputs[0][key]), (j, key)
        kb, vb = R.sorted_keys(frb, j)
        ks, vs = R.sorted_keys(fr1, 0, count=k1)
        assert np.array_equal(kb, ks) and np.array_equal(vb, vs), j
        say(f"  frame {j}: {k1} pairs, identical")
