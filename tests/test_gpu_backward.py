"""Backward-pass parity of the HIP adjoint (through the C ABI and the
torch.autograd.Function) against the FP64 oracle's adjoint, and against
central finite differences of the oracle forward on the 2k-Gaussian 64x64
subset of the 500k-Gaussian scene."""

import numpy as np
import pytest

import oracle
import synth
from oracle import backward as OB

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2605_11489_amd import render as R  # noqa: E402
from paper_2605_11489_amd.autograd import rasterize  # noqa: E402

FIELDS = ("means", "log_scales", "quats", "opacity_logits", "sh")


def say(msg):
    print(msg, flush=True)


def gpu_grads(scene, cam, target, w_alpha=None, w_depth=None, bg=(0.0, 0.0, 0.0)):
    ds = R.DeviceScene.from_host(scene)
    params = [t.clone().requires_grad_(True) for t in ds.tensors()]
    rgb, alpha, depth, dcdx, dcdy = rasterize(*params, cam, bg=bg)
    tgt = torch.from_numpy(target).cuda()
    loss = ((rgb - tgt) ** 2).sum()
    if w_alpha is not None:
        loss = loss + (torch.from_numpy(w_alpha).cuda() * alpha).sum()
    if w_depth is not None:
        loss = loss + (torch.from_numpy(w_depth).cuda() * depth).sum()
    loss.backward()
    return {f: p.grad.cpu().numpy().astype(np.float64) for f, p in zip(FIELDS, params)}, rgb.detach().cpu().numpy()


def oracle_grads(scene, cam, target, w_alpha=None, w_depth=None, bg=(0.0, 0.0, 0.0), tiles=None):
    fr = oracle.render_forward(scene, cam, bg=bg, tiles=tiles, composite_all=tiles is None, track=False)
    d_rgb = 2.0 * (fr.image.rgb - target)
    if tiles is not None:
        mask = np.zeros((cam.height, cam.width), dtype=bool)
        P = fr.proj
        for t in tiles:
            tx, ty = t % P.tiles_x, t // P.tiles_x
            mask[ty * 16:(ty + 1) * 16, tx * 16:(tx + 1) * 16] = True
        d_rgb = d_rgb * mask[None]
    g2 = OB.composite_backward(fr, d_rgb, w_alpha, w_depth, tiles=tiles)
    pg = OB.project_backward(scene, cam, fr.proj, g2)
    return {f: getattr(pg, f) for f in FIELDS}, fr


def compare(g, ref, rel=1e-4):
    worst = {}
    for f in FIELDS:
        scale = max(1.0, float(np.abs(ref[f]).max()))
        err = float(np.abs(g[f] - ref[f]).max())
        worst[f] = (err, scale)
        assert err <= rel * scale, (f, err, scale)
    return worst


@pytest.mark.parametrize("seed,deg,bg", [(41, 3, (0.0, 0.0, 0.0)), (42, 1, (0.2, 0.4, 0.6))])
def test_small_scene_matches_oracle_adjoint(seed, deg, bg):
    say(f"case: backward small scene seed={seed} deg={deg}")
    scene = synth.gen_clustered(seed, 600, deg)
    cam = synth.look_at_camera((0.8, -0.4, -3.5), 72, 56)
    rng = np.random.default_rng(seed)
    target = rng.uniform(0, 1, (3, 56, 72)).astype(np.float32)
    w_alpha = rng.normal(size=(56, 72)).astype(np.float32)
    w_depth = (0.1 * rng.normal(size=(56, 72))).astype(np.float32)
    g, _ = gpu_grads(scene, cam, target, w_alpha, w_depth, bg)
    ref, _ = oracle_grads(scene, cam, target, w_alpha.astype(np.float64), w_depth.astype(np.float64), bg)
    worst = compare(g, ref)
    say("  " + ", ".join(f"{k}: {e:.2e}/{s:.2e}" for k, (e, s) in worst.items()))


def c4_subset():
    """First 2,000 Gaussians (index order) of the 500k scene whose tile
    rectangle meets the 64x64 centre crop, rendered on the crop camera."""
    scene, cam = synth.gen_cfg4()
    crop = synth.crop_camera(cam, 448, 238, 64, 64)
    P = oracle.project.project(scene, crop)
    idx = np.nonzero(P.touched > 0)[0][:2000]
    return scene.subset(idx), crop


def test_fd_subset_of_config4():
    say("case: backward on the 2k-Gaussian 64x64 subset of the 500k scene vs oracle adjoint and central FD")
    sub, cam = c4_subset()
    target = synth.gen_target(1, 64, 64)
    g, _ = gpu_grads(sub, cam, target)
    ref, fr = oracle_grads(sub, cam, target)
    worst = compare(g, ref)
    say("  " + ", ".join(f"{k}: {e:.2e}/{s:.2e}" for k, (e, s) in worst.items()))
    # central differences (h = 1e-4, FP64 oracle forward) on sampled parameters
    rng = np.random.default_rng(7)
    h = 1e-4
    checked = 0

    def L(sc):
        f = oracle.render_forward(sc, cam, track=False)
        return float(((f.image.rgb - target) ** 2).sum()), f

    base_n = fr.image.n_contrib.copy()
    base_b = fr.image.blended.copy()
    for field in FIELDS:
        flat = getattr(sub, field).reshape(-1)
        live = np.nonzero(np.abs(ref[field].reshape(-1)) > 1e-3)[0]
        for i in rng.choice(live, size=min(4, live.size), replace=False):
            vals = []
            ok = True
            for sgn in (1, -1):
                sc = sub.copy()
                a = getattr(sc, field).reshape(-1)
                a[i] = np.float32(np.float64(flat[i]) + sgn * h)
                Lv, f = L(sc)
                if not (np.array_equal(f.image.n_contrib, base_n) and np.array_equal(f.image.blended, base_b)):
                    ok = False
                    break
                vals.append((Lv, float(np.float64(a[i]) - np.float64(flat[i]))))
            if not ok:
                continue
            fd = (vals[0][0] - vals[1][0]) / (vals[0][1] - vals[1][1])
            gv = g[field].reshape(-1)[i]
            assert abs(fd - gv) <= 2e-3 * max(1.0, abs(fd)), (field, i, fd, gv)
            checked += 1
    say(f"  FD-checked parameters: {checked}")
    assert checked >= 10


def test_full_size_config4_sampled_tiles():
    say("case: backward at full size (500k Gaussians, 960x540), loss restricted to sampled tiles")
    scene, cam = synth.gen_cfg4()
    target = synth.gen_target(1, 540, 960)
    rng = np.random.default_rng(3)
    tiles = sorted(rng.choice(2040, 6, replace=False).tolist())
    mask = np.zeros((540, 960), dtype=np.float32)
    for t in tiles:
        tx, ty = t % 60, t // 60
        mask[ty * 16:(ty + 1) * 16, tx * 16:(tx + 1) * 16] = 1.0
    ds = R.DeviceScene.from_host(scene)
    params = [t.clone().requires_grad_(True) for t in ds.tensors()]
    rgb, alpha, depth, _, _ = rasterize(*params, cam)
    m = torch.from_numpy(mask).cuda()
    loss = (((rgb - torch.from_numpy(target).cuda()) ** 2) * m).sum()
    loss.backward()
    g = {f: p.grad.cpu().numpy().astype(np.float64) for f, p in zip(FIELDS, params)}
    ref, _ = oracle_grads(scene, cam, target, tiles=tiles)
    worst = compare(g, ref)
    say("  " + ", ".join(f"{k}: {e:.2e}/{s:.2e}" for k, (e, s) in worst.items()))
    for f in FIELDS:
        assert np.isfinite(g[f]).all()


@pytest.mark.parametrize("seed,deg,W,H", [(43, 0, 37, 23), (44, 2, 53, 41)])
def test_ragged_raster_degrees_0_and_2(seed, deg, W, H):
    """Degree 0 (3 coefficients) and degree 2 (27: not a multiple of 4, so the
    coefficient gradients move as scalars) on rasters whose last tile row and
    column are partial, with alpha and depth terms in the loss."""
    say(f"case: backward ragged {W}x{H} seed={seed} deg={deg}")
    scene = synth.random_scene_small(seed, 400, deg)
    cam = synth.identity_camera(W, H)
    rng = np.random.default_rng(seed)
    target = rng.uniform(0, 1, (3, H, W)).astype(np.float32)
    w_alpha = rng.normal(size=(H, W)).astype(np.float32)
    w_depth = (0.1 * rng.normal(size=(H, W))).astype(np.float32)
    g, _ = gpu_grads(scene, cam, target, w_alpha, w_depth, (0.1, 0.2, 0.3))
    ref, _ = oracle_grads(scene, cam, target, w_alpha.astype(np.float64), w_depth.astype(np.float64),
                          (0.1, 0.2, 0.3))
    worst = compare(g, ref)
    say("  " + ", ".join(f"{k}: {e:.2e}/{s:.2e}" for k, (e, s) in worst.items()))
    assert max(float(np.abs(ref[f]).max()) for f in FIELDS) > 0.0


def test_nothing_visible_gives_zero_gradients():
    say("case: backward with every Gaussian behind the camera")
    scene = synth.random_scene_small(45, 300, 3, lo=(-1.0, -1.0, -6.0), hi=(1.0, 1.0, -2.0))
    cam = synth.identity_camera(64, 48)
    target = np.full((3, 48, 64), 0.5, dtype=np.float32)
    g, rgb = gpu_grads(scene, cam, target)
    assert np.all(rgb == 0.0)
    for f in FIELDS:
        assert np.all(g[f] == 0.0), f


def test_backward_accumulates_into_gradients():
    """Two backward calls on the same buffers add up (the buffers are not
    cleared by the library): the second result is twice the first up to the
    float-atomic summation order."""
    import ctypes as C
    from paper_2605_11489_amd import abi
    say("case: backward called twice accumulates")
    scene = synth.random_scene_small(46, 500, 3)
    cam = synth.identity_camera(80, 64)
    ds = R.DeviceScene.from_host(scene)
    out = R.alloc_outputs(cam.width, cam.height)
    opts = R.opts_struct()
    fr = R.render_batch([(ds, cam, opts, out)], with_backward=True)
    rc, _ = R.forward_status(fr)
    assert rc == 0
    g_rgb = torch.from_numpy(np.random.default_rng(46).normal(size=(3, 64, 80)).astype(np.float32)).cuda()
    grads = [torch.zeros_like(t) for t in ds.tensors()]
    gs = abi.gs_grads(*[t.data_ptr() for t in grads])
    sc, cs, outs = ds.c_struct(), R.camera_struct(cam), R.outputs_struct(out)

    def call():
        abi.check(abi.gs_render_backward(C.byref(sc), C.byref(cs), C.byref(opts), C.byref(outs),
                                         fr.workspace.data_ptr(), fr.workspace.numel(), fr.key_capacity,
                                         g_rgb.data_ptr(), None, None, C.byref(gs), R.current_stream_ptr()))
        torch.cuda.synchronize()
        return [t.cpu().numpy().astype(np.float64) for t in grads]

    one = call()
    two = call()
    for f, a, b in zip(FIELDS, one, two):
        scale = max(1.0, float(np.abs(a).max()))
        assert float(np.abs(b - 2.0 * a).max()) <= 1e-5 * scale, f
        assert float(np.abs(a).max()) > 0.0, f


@pytest.mark.parametrize("mode", [1, 2])
def test_backward_after_shorter_lists(mode):
    """The backward pass over the lists of the opacity-aware (box or exact
    ellipse) overlap gives the square lists' gradients: the dropped pairs
    never blend, so only the float-atomic summation order differs."""
    import ctypes as C
    from paper_2605_11489_amd import abi
    say(f"case: backward after overlap mode {mode} vs the square")
    scene = synth.random_scene_small(47, 600, 3)
    cam = synth.identity_camera(90, 70)
    ds = R.DeviceScene.from_host(scene)
    g_rgb = torch.from_numpy(np.random.default_rng(47).normal(size=(3, 70, 90)).astype(np.float32)).cuda()
    res = {}
    for m in (0, mode):
        out = R.alloc_outputs(cam.width, cam.height)
        opts = R.opts_struct(overlap=m)
        fr = R.render_batch([(ds, cam, opts, out)], with_backward=True)
        rc, k = R.forward_status(fr)
        assert rc == 0
        grads = [torch.zeros_like(t) for t in ds.tensors()]
        gs = abi.gs_grads(*[t.data_ptr() for t in grads])
        sc, cs, outs = ds.c_struct(), R.camera_struct(cam), R.outputs_struct(out)
        abi.check(abi.gs_render_backward(C.byref(sc), C.byref(cs), C.byref(opts), C.byref(outs),
                                         fr.workspace.data_ptr(), fr.workspace.numel(), fr.key_capacity,
                                         g_rgb.data_ptr(), None, None, C.byref(gs), R.current_stream_ptr()))
        torch.cuda.synchronize()
        res[m] = ([t.cpu().numpy().astype(np.float64) for t in grads], k)
    assert res[mode][1] < res[0][1]
    for f, a, b in zip(FIELDS, res[0][0], res[mode][0]):
        scale = max(1.0, float(np.abs(a).max()))
        assert float(np.abs(a - b).max()) <= 1e-5 * scale, f


def test_autograd_workspace_growth_and_two_live_graphs():
    """The autograd Function keeps workspaces per (device, n, degree, raster)
    and grows their key capacity when a frame needs more pairs: a far view
    sets a small capacity, a near view of the same class outgrows it and is
    re-run.  Two graphs alive at once (two forwards, then both backwards)
    hold separate workspaces.  Every gradient matches the FP64 adjoint."""
    say("case: autograd workspace reuse, growth and two live graphs")
    scene = synth.gen_clustered(43, 600, 2)
    far = synth.look_at_camera((0.4, -0.2, -7.0), 72, 56)
    near = synth.look_at_camera((0.3, 0.2, -2.6), 72, 56)
    rng = np.random.default_rng(43)
    target = rng.uniform(0, 1, (3, 56, 72)).astype(np.float32)
    # far then near: the near frame needs more pairs than the far one left room for
    g_far, _ = gpu_grads(scene, far, target)
    g_near, _ = gpu_grads(scene, near, target)
    for cam, g in ((far, g_far), (near, g_near)):
        ref, _ = oracle_grads(scene, cam, target)
        compare(g, ref)
    # two graphs alive at once: both backwards after both forwards
    ds = R.DeviceScene.from_host(scene)
    tgt = torch.from_numpy(target).cuda()
    pa = [t.clone().requires_grad_(True) for t in ds.tensors()]
    pb = [t.clone().requires_grad_(True) for t in ds.tensors()]
    la = ((rasterize(*pa, near)[0] - tgt) ** 2).sum()
    lb = ((rasterize(*pb, far)[0] - tgt) ** 2).sum()
    lb.backward()
    la.backward()
    for params, g in ((pa, g_near), (pb, g_far)):
        for f, p in zip(FIELDS, params):
            got = p.grad.cpu().numpy().astype(np.float64)
            scale = max(1.0, float(np.abs(g[f]).max()))
            assert np.abs(got - g[f]).max() <= 1e-5 * scale, f


def test_checked_forward_reports_capacity_and_reruns():
    """gs_render_forward_checked with too small a key capacity returns
    GS_ERR_CAPACITY and the pair count; called again with that capacity it
    renders the same frame as gs_render_forward_batch sized exactly."""
    from paper_2605_11489_amd import abi
    say("case: checked forward, capacity too small then exact")
    scene = synth.gen_clustered(44, 3000, 3)
    cam = synth.look_at_camera((0.5, -0.3, -3.2), 97, 61)
    ds = R.DeviceScene.from_host(scene)
    opts = R.opts_struct(bg=(0.2, 0.3, 0.4))
    out = R.alloc_outputs(cam.width, cam.height)
    jobs = R.make_jobs([(ds, cam, opts, out)])
    L = R.layout_for(jobs, 1, 10)
    ws = R.alloc_workspace(L.total_bytes)
    rc, need = R.render_checked(jobs, 1, ws, 10)
    assert rc == abi.GS_ERR_CAPACITY and need > 10
    L = R.layout_for(jobs, 1, need)
    ws = R.alloc_workspace(L.total_bytes)
    rc, need2 = R.render_checked(jobs, 1, ws, need)
    assert rc == abi.GS_OK and need2 == need
    ref = R.render(ds, cam, bg=(0.2, 0.3, 0.4))
    rc, k = R.forward_status(ref)
    assert rc == 0 and k == need
    for key in ("rgb", "alpha", "depth", "dcdx", "dcdy", "final_T", "n_contrib"):
        assert torch.equal(out[key], ref.outputs[0][key]), key


def test_autograd_deferred_check_raises_on_overflow():
    """A graph-building call launches with the cached capacity and checks its
    pair count in the backward: a frame that outgrows it raises
    GS_ERR_CAPACITY there (after growing the capacity), and the next step
    runs with room to spare and gives the oracle's gradients."""
    from paper_2605_11489_amd import abi
    from paper_2605_11489_amd import autograd as AG
    say("case: autograd deferred pair-count check, overflow then rerun")
    scene = synth.gen_clustered(45, 600, 1)
    scene.log_scales += 1.5          # large splats: ~1.5k pairs from afar, ~7.2k close up
    far = synth.look_at_camera((0.4, -0.2, -14.0), 160, 120)
    near = synth.look_at_camera((0.3, 0.2, -2.5), 160, 120)
    rng = np.random.default_rng(45)
    target = rng.uniform(0, 1, (3, 120, 160)).astype(np.float32)
    ds = R.DeviceScene.from_host(scene)
    tgt = torch.from_numpy(target).cuda()
    params = [t.clone().requires_grad_(True) for t in ds.tensors()]
    ((rasterize(*params, far)[0] - tgt) ** 2).sum().backward()     # sets a small capacity
    key = (torch.cuda.current_device(), scene.n, scene.sh_degree, 160, 120)
    cap0 = AG._POOL[key].capacity
    for p in params:
        p.grad = None
    loss = ((rasterize(*params, near)[0] - tgt) ** 2).sum()
    with pytest.raises(abi.GsError) as ei:
        loss.backward()
    assert ei.value.code == abi.GS_ERR_CAPACITY
    assert AG._POOL[key].capacity > cap0
    for p in params:
        p.grad = None
    ((rasterize(*params, near)[0] - tgt) ** 2).sum().backward()
    ref, _ = oracle_grads(scene, near, target)
    compare({f: p.grad.cpu().numpy().astype(np.float64) for f, p in zip(FIELDS, params)}, ref)


def test_backward_overwrite_mode_equals_accumulate_from_zero():
    """grads->overwrite = 1 writes every Gaussian's gradients (zeros for
    those that reach no tile) into arrays holding garbage: the result equals
    the accumulating call on zeroed arrays (to the rounding of the float
    atomics' order)."""
    say("case: backward overwrite mode vs accumulation into zeros")
    scene = synth.gen_clustered(46, 2000, 3)
    cam = synth.look_at_camera((0.6, -0.3, -3.0), 83, 59)
    ds = R.DeviceScene.from_host(scene)
    fr = R.render(ds, cam, with_backward=True)
    assert R.forward_status(fr)[0] == 0
    rng = np.random.default_rng(46)
    g_rgb = torch.from_numpy(rng.normal(size=(3, 59, 83)).astype(np.float32)).cuda()
    acc = [torch.zeros_like(t) for t in ds.tensors()]
    R.render_backward(fr, g_rgb, acc)
    torch.cuda.synchronize()
    put = [torch.full_like(t, float("nan")) for t in ds.tensors()]
    R.render_backward(fr, g_rgb, put, overwrite=True)
    torch.cuda.synchronize()
    for f, a, b in zip(FIELDS, acc, put):
        assert torch.isfinite(b).all(), f
        diff = (a - b).abs().max().item()
        assert diff <= 1e-6 * max(1.0, a.abs().max().item()), (f, diff)
    n_untouched = int((acc[3] == 0).sum().item())
    say(f"  Gaussians with zero opacity gradient: {n_untouched}")
