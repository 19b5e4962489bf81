"""Pins of the motion-vector and warping oracle (Sec. 4.2, Eq. 12-13) against
closed forms: a fronto-parallel plane seen from a camera translated sideways
(uniform V = -fx b / z0; an integer shift copies pixels exactly, gradients
unchanged) and from a camera moved forward (V = (s - 1)(x - c), gradients
scaled by 1 / s), background pixels that do not move, and the z-buffer
against an independent lexsort of all landings."""

import numpy as np

import synth
from oracle import warp as Wp


def cam_at(t, W, H, fx=40.0):
    c = synth.Camera(R_wc=np.eye(3).reshape(-1).tolist(), t=list(map(float, t)), fx=fx, fy=fx, cx=W / 2, cy=H / 2,
                     width=W, height=H)
    return c


def plane(W, H, z0, rng):
    alpha = np.ones((H, W), np.float32)
    depth = np.full((H, W), z0, np.float32)
    rgb, gx, gy = synth.image_fields(int(rng.integers(1 << 30)), W, H)
    return alpha, depth, rgb, gx, gy


def test_sideways_translation_integer_shift():
    W, H, z0, fx = 24, 16, 4.0, 40.0
    b = 0.3          # fx b / z0 = 3 pixels
    rng = np.random.default_rng(0)
    alpha, depth, rgb, gx, gy = plane(W, H, z0, rng)
    src, dst = cam_at((0, 0, 0), W, H, fx), cam_at((-b, 0, 0), W, H, fx)
    out = Wp.warp(src, dst, rgb, alpha, depth, gx, gy, W, H)
    assert np.allclose(out["motion"][0], -3.0, atol=1e-12) and np.allclose(out["motion"][1], 0.0, atol=1e-12)
    # destination column i holds source column i + 3; the last 3 columns are holes
    assert np.array_equal(out["rgb"][:, :, :W - 3], rgb[:, :, 3:].astype(np.float64))
    assert np.all(out["weight"][:, W - 3:] == 0) and np.all(out["weight"][:, :W - 3] == 1)
    assert np.allclose(out["dcdx"][:, :, :W - 3], gx[:, :, 3:], atol=1e-12)
    assert np.allclose(out["dcdy"][:, :, :W - 3], gy[:, :, 3:], atol=1e-12)
    assert np.allclose(out["depth"][:, :W - 3], z0)


def test_forward_motion_scales_gradients():
    W, H, z0, d, fx = 20, 14, 4.0, 1.0, 30.0
    rng = np.random.default_rng(1)
    alpha, depth, rgb, gx, gy = plane(W, H, z0, rng)
    src, dst = cam_at((0, 0, 0), W, H, fx), cam_at((0, 0, -d), W, H, fx)
    out = Wp.warp(src, dst, rgb, alpha, depth, gx, gy, W, H)
    s = z0 / (z0 - d)
    U, V = np.meshgrid(np.arange(W) + 0.5, np.arange(H) + 0.5)
    assert np.allclose(out["motion"][0], (U - W / 2) * (s - 1), atol=1e-9)
    assert np.allclose(out["motion"][1], (V - H / 2) * (s - 1), atol=1e-9)
    src_idx = out["source"]
    hit = src_idx >= 0
    sj, si = np.divmod(src_idx[hit], W)
    # the Jacobian of a linear motion field is exact under central differences
    assert np.allclose(out["dcdx"][:, hit], gx[:, sj, si] / s, atol=1e-12)
    assert np.allclose(out["dcdy"][:, hit], gy[:, sj, si] / s, atol=1e-12)
    assert np.allclose(out["depth"][hit], z0 - d)


def test_background_does_not_move():
    W, H = 10, 8
    rng = np.random.default_rng(2)
    alpha, depth, rgb, gx, gy = plane(W, H, 3.0, rng)
    alpha[:, :5] = 0.0
    depth[:, :5] = 0.0
    src, dst = cam_at((0, 0, 0), W, H), cam_at((-0.1, 0.05, 0), W, H)
    out = Wp.warp(src, dst, rgb, alpha, depth, gx, gy, W, H)
    assert np.all(out["motion"][:, :, :5] == 0.0)
    sj, si = np.divmod(out["source"][out["source"] >= 0], W)
    assert np.all(si >= 5)


def test_zbuffer_against_lexsort():
    """Near patch over far background, camera moved sideways: the winner of
    every destination pixel is the minimum (float32 z', source index) among
    the pixels landing there."""
    W, H = 30, 20
    rng = np.random.default_rng(3)
    alpha = np.ones((H, W), np.float32)
    depth = np.full((H, W), 6.0, np.float32)
    depth[5:12, 8:18] = 2.0
    rgb, gx, gy = synth.image_fields(4, W, H)
    src, dst = cam_at((0, 0, 0), W, H), cam_at((-0.25, 0.0, 0.0), W, H)
    out = Wp.warp(src, dst, rgb, alpha, depth, gx, gy, W, H)
    V, zd, geom, ok, ud, vd = Wp.motion(src, dst, alpha, depth)
    ti, tj = np.floor(ud).astype(int), np.floor(vd).astype(int)
    land = ok & (ti >= 0) & (ti < W) & (tj >= 0) & (tj < H)
    k = (tj * W + ti)[land]
    z = zd[land].astype(np.float32)
    idx = np.arange(H * W).reshape(H, W)[land]
    order = np.lexsort((idx, z, k))
    first = np.ones(order.size, bool)
    first[1:] = k[order][1:] != k[order][:-1]
    expect = np.full(H * W, -1)
    expect[k[order][first]] = idx[order][first]
    assert np.array_equal(out["source"].reshape(-1), expect)
    # occlusion happened: some destination pixels had several candidates
    assert np.bincount(k).max() >= 2


def test_roll_rotates_gradients():
    """Destination camera rolled by theta about its optical axis, plane at z0:
    the image rotates about the principal point, dV/dx = Rot - I, so the
    warped gradient is Rot applied to the source gradient (a transposed
    Jacobian would rotate it the other way)."""
    W, H, z0, fx, th = 26, 26, 3.0, 35.0, 0.2
    rng = np.random.default_rng(5)
    alpha, depth, rgb, gx, gy = plane(W, H, z0, rng)
    c, s = np.cos(th), np.sin(th)
    Rz = np.array([[c, -s, 0.0], [s, c, 0.0], [0.0, 0.0, 1.0]])
    src = cam_at((0, 0, 0), W, H, fx)
    dst = synth.Camera(R_wc=Rz.reshape(-1).tolist(), t=[0.0, 0.0, 0.0], fx=fx, fy=fx, cx=W / 2, cy=H / 2,
                       width=W, height=H)
    out = Wp.warp(src, dst, rgb, alpha, depth, gx, gy, W, H)
    U, V = np.meshgrid(np.arange(W) + 0.5, np.arange(H) + 0.5)
    du, dv = U - W / 2, V - H / 2
    assert np.allclose(out["motion"][0], c * du - s * dv - du, atol=1e-9)
    assert np.allclose(out["motion"][1], s * du + c * dv - dv, atol=1e-9)
    hit = out["source"] >= 0
    sj, si = np.divmod(out["source"][hit], W)
    # interior sources only (central differences on both sides)
    inner = (si > 0) & (si < W - 1) & (sj > 0) & (sj < H - 1)
    gxs, gys = gx[:, sj, si][:, inner], gy[:, sj, si][:, inner]
    assert np.allclose(out["dcdx"][:, hit][:, inner], c * gxs - s * gys, atol=1e-9)
    assert np.allclose(out["dcdy"][:, hit][:, inner], s * gxs + c * gys, atol=1e-9)


def test_normals_follow_the_camera_rotation():
    """Normals are re-expressed in the destination camera's axes: unchanged
    (bit for bit) under a pure translation; under a yaw of the destination
    by theta, n' = Ry(theta) n, checked against scipy; holes stay 0."""
    from scipy.spatial.transform import Rotation
    W, H, z0 = 30, 20, 4.0
    rng = np.random.default_rng(6)
    alpha, depth, rgb, gx, gy = plane(W, H, z0, rng)
    nrm = rng.normal(size=(3, H, W)).astype(np.float32)
    src = cam_at((0, 0, 0), W, H)
    out = Wp.warp(src, cam_at((-0.1, 0.02, 0.1), W, H), rgb, alpha, depth, gx, gy, W, H, normal=nrm)
    hit = out["source"] >= 0
    sj, si = np.divmod(out["source"][hit], W)
    assert np.array_equal(out["normal"][:, hit], nrm[:, sj, si].astype(np.float64))
    assert np.all(out["normal"][:, ~hit] == 0)
    th = 0.05
    Ry = Rotation.from_euler("y", th).as_matrix()
    dst = synth.Camera(R_wc=Ry.reshape(-1).tolist(), t=[0.0, 0.0, 0.0], fx=40.0, fy=40.0, cx=W / 2, cy=H / 2,
                       width=W, height=H)
    out = Wp.warp(src, dst, rgb, alpha, depth, gx, gy, W, H, normal=nrm)
    hit = out["source"] >= 0
    sj, si = np.divmod(out["source"][hit], W)
    assert hit.mean() > 0.5
    assert np.allclose(out["normal"][:, hit], Ry @ nrm[:, sj, si].astype(np.float64), atol=1e-12)


def test_fold_has_no_gradient_and_sampled_jacobian_agrees():
    """Where I + dV/dx is singular (the motion field folds) the warped
    gradient is zero; the Jacobian evaluated at sampled pixels equals the
    full field's at those pixels."""
    g = np.array([0.3, -0.2, 0.1])
    gx, gy = Wp.warp_gradient(-np.eye(2), g, 2 * g)
    assert np.all(gx == 0) and np.all(gy == 0)
    gx, gy = Wp.warp_gradient(np.array([[0.0, 0.0], [0.0, -1.0]]), g, 2 * g)
    assert np.all(gx == 0) and np.all(gy == 0)
    W, H = 23, 17
    alpha, depth, _, _, _ = synth.frame_fields(9, W, H)
    src, dst = cam_at((0, 0, 0), W, H), cam_at((-0.2, 0.1, 0.3), W, H)
    V, zd, geom, ok, ud, vd = Wp.motion(src, dst, alpha, depth)
    J = Wp.jacobian(V, geom)
    rng = np.random.default_rng(0)
    pj, pi = rng.integers(0, H, 50), rng.integers(0, W, 50)
    assert np.array_equal(Wp.jacobian(V, geom, points=(pj, pi)), J[pj, pi])
