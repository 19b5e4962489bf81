"""Pins of the oracle's normal maps (N and Nv, Sec. 4.1 and 4.2; shortest-axis
normals blended like colour, the RaDe-GS rendering named in Sec. 5.1)
against closed forms: a disc facing the camera, a rotated ellipsoid whose
normal is a column of scipy's rotation matrix, the two-layer stack, many
layers sharing one normal (N = alpha n by the telescoping of the weights),
and the tie and orientation rules.  CPU only."""

import math

import numpy as np
from scipy.spatial.transform import Rotation

import oracle
import synth
from oracle import conventions as cv
from oracle.composite import normal_view


def scene_of(means, log_scales, quats, logits, degree=0):
    n = len(means)
    shc = np.zeros((n, (degree + 1) ** 2, 3), dtype=np.float32)
    return synth.Scene(np.asarray(means, np.float32), np.asarray(log_scales, np.float32),
                       np.asarray(quats, np.float32), np.asarray(logits, np.float32), shc, degree)


def ray_cos(cam, ix, iy):
    """cos of the angle between the optical axis and pixel (ix, iy)'s ray."""
    rx = (ix + 0.5 - cam.cx) / cam.fx
    ry = (iy + 0.5 - cam.cy) / cam.fy
    return 1.0 / math.sqrt(rx * rx + ry * ry + 1.0)


def test_disc_facing_the_camera():
    """Thin along z, identity rotation, camera looking down +z: n = (0, 0, -1)
    and, at every pixel, N = alpha n and Nv = alpha cos(ray angle)."""
    cam = synth.identity_camera(48, 32)
    sc = scene_of([[0.05, -0.03, 3.0]], [[-1.8, -2.1, -7.0]], [[1, 0, 0, 0]], [1.2])
    fr = oracle.render_forward(sc, cam)
    assert np.array_equal(fr.proj.normal[0], [0.0, 0.0, -1.0])
    img = fr.image
    for iy in range(32):
        for ix in range(48):
            a = img.alpha[iy, ix]
            assert np.allclose(img.normal[:, iy, ix], [0.0, 0.0, -a], atol=1e-15)
            assert abs(img.nv[iy, ix] - a * ray_cos(cam, ix, iy)) < 1e-14
    assert img.alpha.max() > 0.5


def test_rotated_ellipsoid_normal_is_scipy_column():
    """Random rotations and shortest axes under a look-at camera: the normal
    is the shortest axis from scipy's quaternion -> matrix (an independent
    route), rotated into the camera and flipped towards it."""
    rng = np.random.default_rng(3)
    cam = synth.look_at_camera((1.0, -0.5, -4.0), 64, 64)
    n = 200
    q = rng.normal(size=(n, 4)).astype(np.float32)
    ls = rng.normal(-3.0, 0.6, size=(n, 3)).astype(np.float32)
    means = rng.uniform(-0.6, 0.6, size=(n, 3)).astype(np.float32)
    fr = oracle.render_forward(scene_of(means, ls, q, np.zeros(n)), cam, composite_all=False)
    R = np.asarray(cam.R_wc)
    for g in range(n):
        w, x, y, z = q[g].astype(np.float64)
        Rq = Rotation.from_quat([x, y, z, w]).as_matrix()
        k = int(np.argmin(ls[g]))
        nc = R @ Rq[:, k]
        pc = R @ means[g].astype(np.float64) + np.asarray(cam.t)
        if nc @ pc > 0:
            nc = -nc
        assert np.allclose(fr.proj.normal[g], nc, atol=1e-12), g
        assert abs(np.linalg.norm(fr.proj.normal[g]) - 1.0) < 1e-12
        assert fr.proj.normal[g] @ pc <= 0.0


def test_two_layer_stack():
    """Two tilted discs at one pixel: N = a1 n1 + (1 - a1) a2 n2 with the
    alphas from the Gaussians' closed form."""
    cam = synth.identity_camera(32, 32)
    r1 = Rotation.from_euler("x", 0.4)
    r2 = Rotation.from_euler("y", -0.7)
    q1 = np.roll(r1.as_quat(), 1)   # scipy (x, y, z, w) -> (w, x, y, z)
    q2 = np.roll(r2.as_quat(), 1)
    sc = scene_of([[0.01, 0.0, 2.0], [-0.02, 0.01, 3.0]], [[-2.4, -2.6, -6.0], [-6.5, -2.0, -2.2]],
                  [q1, q2], [0.3, 1.1])
    fr = oracle.render_forward(sc, cam)
    P = fr.proj
    ix, iy = 17, 14
    n_exp = [r1.as_matrix()[:, 2], r2.as_matrix()[:, 0]]
    al = []
    for g in range(2):
        if n_exp[g] @ np.array([P.x[g], P.y[g], P.z[g]]) > 0:
            n_exp[g] = -n_exp[g]
        assert np.allclose(P.normal[g], n_exp[g], atol=1e-7)   # float32 quaternion input
        cov = np.array([[P.cov2d[g, 0], P.cov2d[g, 1]], [P.cov2d[g, 1], P.cov2d[g, 2]]])
        d = np.array([P.u[g] - (ix + 0.5), P.v[g] - (iy + 0.5)])
        a = P.opacity[g] * math.exp(-0.5 * d @ np.linalg.inv(cov) @ d)
        assert cv.ALPHA_MIN < a < cv.ALPHA_MAX
        al.append(a)
    a1, a2 = al
    N = a1 * P.normal[0] + (1 - a1) * a2 * P.normal[1]
    assert np.allclose(fr.image.normal[:, iy, ix], N, atol=1e-13)
    assert abs(fr.image.nv[iy, ix] - normal_view(N, cam, ix, iy)) < 1e-13


def test_shared_normal_telescopes_to_alpha():
    """Many overlapping discs that all face the camera: the blend weights sum
    to alpha, so N = alpha (0, 0, -1) at every pixel."""
    rng = np.random.default_rng(5)
    n = 400
    cam = synth.identity_camera(48, 48)
    means = np.stack([rng.uniform(-0.5, 0.5, n), rng.uniform(-0.5, 0.5, n), rng.uniform(2.0, 5.0, n)], axis=1)
    ls = np.stack([rng.uniform(-3.5, -2.5, n), rng.uniform(-3.5, -2.5, n), np.full(n, -8.0)], axis=1)
    fr = oracle.render_forward(scene_of(means, ls, np.tile([1.0, 0, 0, 0], (n, 1)), rng.normal(0, 1, n)), cam)
    img = fr.image
    assert np.allclose(img.normal[2], -img.alpha, atol=1e-13)
    assert np.all(img.normal[:2] == 0.0)
    assert img.alpha.max() > 0.9 and fr.image.n_contrib.max() > 5


def test_ties_take_the_first_axis_and_face_the_camera():
    """Equal scales: the first axis (x) is the normal; a Gaussian right of
    the optical axis gets (-1, 0, 0), one on the left (1, 0, 0)."""
    cam = synth.identity_camera(32, 32)
    sc = scene_of([[0.2, 0.0, 3.0], [-0.2, 0.0, 3.0]], [[-2.0] * 3] * 2, [[1, 0, 0, 0]] * 2, [0.0, 0.0])
    P = oracle.render_forward(sc, cam, composite_all=False).proj
    assert np.array_equal(P.normal[0], [-1.0, 0.0, 0.0])
    assert np.array_equal(P.normal[1], [1.0, 0.0, 0.0])
