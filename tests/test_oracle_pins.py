"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics
(closed forms, identities, brute force, library routines the oracle does not
use, finite differences).  CPU only."""

import math

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

import oracle
import synth
from oracle import binning, brute, composite, conventions as cv, sh
from oracle.project import project, quat_to_rot


def one_gaussian_scene(mean, log_scale, quat, logit, rgb, degree=0):
    k = (degree + 1) ** 2
    shc = np.zeros((1, k, 3), dtype=np.float32)
    shc[0, 0, :] = (np.asarray(rgb) - 0.5) / synth.SH_C0_INPUT
    return synth.Scene(np.array([mean], dtype=np.float32),
                       np.array([log_scale], dtype=np.float32),
                       np.array([quat], dtype=np.float32),
                       np.array([logit], dtype=np.float32), shc, degree)


def stack_scene(means, log_scales, quats, logits, rgbs):
    n = len(means)
    shc = np.zeros((n, 1, 3), dtype=np.float32)
    shc[:, 0, :] = (np.asarray(rgbs) - 0.5) / synth.SH_C0_INPUT
    return synth.Scene(np.asarray(means, dtype=np.float32), np.asarray(log_scales, dtype=np.float32),
                       np.asarray(quats, dtype=np.float32), np.asarray(logits, dtype=np.float32), shc, 0)


# ---------------------------------------------------------------- SH basis

def sphere_quadrature(n_theta=24, n_phi=48):
    x, w = np.polynomial.legendre.leggauss(n_theta)        # cos(theta) nodes
    phi = 2 * np.pi * np.arange(n_phi) / n_phi
    ct, ph = np.meshgrid(x, phi, indexing="ij")
    st = np.sqrt(1 - ct ** 2)
    d = np.stack([st * np.cos(ph), st * np.sin(ph), ct], axis=-1).reshape(-1, 3)
    wt = (w[:, None] * np.full(n_phi, 2 * np.pi / n_phi)[None, :]).ravel()
    return d, wt


def test_sh_orthonormal_by_quadrature():
    d, wt = sphere_quadrature()
    Y = sh.basis(d, 3)
    gram = (Y * wt[:, None]).T @ Y
    assert np.abs(gram - np.eye(16)).max() < 1e-12


def test_sh_addition_theorem():
    # sum_m Y_lm(a) Y_lm(b) = (2l+1)/(4 pi) P_l(a.b): fixes each band's normalisation
    rng = np.random.default_rng(3)
    a = rng.normal(size=(50, 3)); a /= np.linalg.norm(a, axis=1, keepdims=True)
    b = rng.normal(size=(50, 3)); b /= np.linalg.norm(b, axis=1, keepdims=True)
    Ya, Yb = sh.basis(a, 3), sh.basis(b, 3)
    cos = (a * b).sum(1)
    for l in range(4):
        sl = slice(l * l, (l + 1) ** 2)
        lhs = (Ya[:, sl] * Yb[:, sl]).sum(1)
        rhs = (2 * l + 1) / (4 * np.pi) * np.polynomial.legendre.legval(cos, [0] * l + [1])
        assert np.abs(lhs - rhs).max() < 1e-12


def test_sh_band1_is_linear_with_cs_phase():
    # reading: Condon-Shortley phase, order m=-1,0,1 -> (-y, z, -x) sqrt(3/4pi)
    d = np.array([[0.0, 0.0, 1.0], [1.0, 0.0, 0.0], [0.0, 1.0, 0.0]])
    Y = sh.basis(d, 1)
    c1 = math.sqrt(3 / (4 * math.pi))
    assert np.allclose(Y[:, 1:], [[0, c1, 0], [0, 0, -c1], [-c1, 0, 0]], atol=1e-15)


def test_sh_basis_matches_scipy_condon_shortley_real_harmonics():
    # All 16 functions, signs and order included, against scipy's complex
    # harmonics (which carry the Condon-Shortley phase), combined into the real
    # basis of the reading: sqrt(2) Re Y_l^m for m > 0, Y_l^0, and
    # sqrt(2) Im Y_l^|m| for m < 0, ordered m = -l..l.  A flipped sign or a
    # swapped pair of functions fails here (orthonormality and the addition
    # theorem cannot see either).
    from scipy.special import sph_harm_y
    rng = np.random.default_rng(31)
    d = rng.normal(size=(400, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    theta = np.arccos(np.clip(d[:, 2], -1.0, 1.0))     # polar angle from +z
    phi = np.arctan2(d[:, 1], d[:, 0])                  # azimuth from +x towards +y
    ref = []
    for l in range(4):
        for m in range(-l, l + 1):
            y = sph_harm_y(l, abs(m), theta, phi)
            if m > 0:
                ref.append(math.sqrt(2.0) * y.real)
            elif m < 0:
                ref.append(math.sqrt(2.0) * y.imag)
            else:
                ref.append(y.real)
    ref = np.stack(ref, axis=1)
    assert np.abs(sh.basis(d, 3) - ref).max() < 1e-12


def test_degree1_colour_uses_the_world_direction_from_camera_to_mean():
    # Colour of a Gaussian with only band-1 coefficients f_-1, f_0, f_1 (per
    # channel) under a rotated look-at camera: 0.5 + sqrt(3/(4 pi)) (-f_-1 d_y
    # + f_0 d_z - f_1 d_x), d the unit vector from the eye to the mean in world
    # axes.  A reversed direction, or one taken in camera axes, fails.
    rng = np.random.default_rng(32)
    n = 64
    eye = np.array([2.1, -1.3, -3.0])
    cam = synth.look_at_camera(eye, 64, 48, target=(0.2, 0.1, 0.3))
    means = rng.uniform(-0.8, 0.8, size=(n, 3)).astype(np.float32)
    shc = np.zeros((n, 4, 3), dtype=np.float32)
    shc[:, 1:, :] = rng.normal(0.0, 1.0, size=(n, 3, 3))
    scene = synth.Scene(means, np.full((n, 3), -3.0, np.float32),
                        np.tile(np.array([[1.0, 0.0, 0.0, 0.0]], np.float32), (n, 1)),
                        np.zeros(n, np.float32), shc, 1)
    P = project(scene, cam)
    d = means.astype(np.float64) - eye
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    f = shc.astype(np.float64)
    c1 = math.sqrt(3.0 / (4.0 * math.pi))
    want = 0.5 + c1 * (-f[:, 1, :] * d[:, 1:2] + f[:, 2, :] * d[:, 2:3] - f[:, 3, :] * d[:, 0:1])
    assert np.abs(P.rgb_raw - want).max() < 1e-12


def test_sh_gradient_matches_finite_differences():
    rng = np.random.default_rng(4)
    d = rng.normal(size=(20, 3))
    G = sh.basis_grad(d, 3)
    h = 1e-6
    for j in range(3):
        e = np.zeros(3); e[j] = h
        fd = (sh.basis(d + e, 3) - sh.basis(d - e, 3)) / (2 * h)
        assert np.abs(fd - G[:, :, j]).max() < 1e-7


# ---------------------------------------------------------------- projection

def test_quaternion_rotation_matches_scipy():
    rng = np.random.default_rng(5)
    q = rng.normal(size=(100, 4)) * rng.uniform(0.2, 3.0, size=(100, 1))   # not unit
    R, _ = quat_to_rot(q.astype(np.float32))
    qf = q.astype(np.float32).astype(np.float64)
    ref = Rotation.from_quat(np.stack([qf[:, 1], qf[:, 2], qf[:, 3], qf[:, 0]], 1)).as_matrix()
    assert np.abs(R - ref).max() < 1e-12


@pytest.mark.parametrize("pos", [(0.0, 0.0, 3.0), (0.4, -0.3, 2.5), (-0.7, 0.6, 5.0)])
def test_isotropic_gaussian_closed_form(pos):
    # Sigma' = s^2 f^2/Z^2 [[1+X^2/Z^2, XY/Z^2],[XY/Z^2, 1+Y^2/Z^2]] + 0.3 I, for any quaternion
    X, Y, Z = pos
    sig = 0.02
    W = H = 256
    cam = synth.identity_camera(W, H)
    f = cam.fx
    scene = one_gaussian_scene(pos, [math.log(sig)] * 3, [0.3, -0.5, 0.7, 0.2], 0.0, [0.5, 0.5, 0.5])
    P = project(scene, cam)
    X, Y, Z = (float(np.float32(c)) for c in pos)
    s2 = float(np.float32(math.log(sig)))
    s2 = math.exp(s2) ** 2
    k = s2 * f * f / (Z * Z)
    ref = np.array([k * (1 + X * X / (Z * Z)) + cv.DILATION, k * X * Y / (Z * Z), k * (1 + Y * Y / (Z * Z)) + cv.DILATION])
    assert np.allclose(P.cov2d[0], ref, rtol=1e-12, atol=1e-12 * ref.max())
    assert abs(P.u[0] - (f * X / Z + 128)) < 1e-9 and abs(P.v[0] - (f * Y / Z + 128)) < 1e-9
    lam = np.linalg.eigvalsh(np.array([[ref[0], ref[1]], [ref[1], ref[2]]])).max()
    r = math.ceil(3 * math.sqrt(lam))
    assert P.radius[0] == r
    tx0, tx1 = max(0, math.floor((P.u[0] - r) / 16)), min(15, math.floor((P.u[0] + r) / 16))
    ty0, ty1 = max(0, math.floor((P.v[0] - r) / 16)), min(15, math.floor((P.v[0] + r) / 16))
    assert tuple(P.rect[0]) == (tx0, ty0, tx1, ty1)
    assert P.touched[0] == (tx1 - tx0 + 1) * (ty1 - ty0 + 1)
    # same Gaussian, another quaternion: nothing changes
    scene2 = one_gaussian_scene(pos, [math.log(sig)] * 3, [1, 0, 0, 0], 0.0, [0.5, 0.5, 0.5])
    P2 = project(scene2, cam)
    assert np.allclose(P2.cov2d, P.cov2d, rtol=1e-12)


def test_ewa_matches_finite_difference_jacobian_under_a_rotated_camera():
    # independent route: world covariance from scipy rotations, perspective Jacobian by FD
    rng = np.random.default_rng(6)
    scene = synth.gen_clustered(1, 50, 0)
    cam = synth.look_at_camera((1.5, -0.5, -3.5), 320, 240)
    P = project(scene, cam)
    for g in np.nonzero(P.valid)[0][:20]:
        qf = scene.quats[g].astype(np.float64)
        Rq = Rotation.from_quat([qf[1], qf[2], qf[3], qf[0]]).as_matrix()
        S = np.diag(np.exp(scene.log_scales[g].astype(np.float64)) ** 2)
        Sw = Rq @ S @ Rq.T
        Sc = cam.R_wc @ Sw @ cam.R_wc.T
        pc = cam.R_wc @ scene.means[g].astype(np.float64) + cam.t

        def pi(p):
            return np.array([cam.fx * p[0] / p[2] + cam.cx, cam.fy * p[1] / p[2] + cam.cy])
        Jfd = np.stack([(pi(pc + e) - pi(pc - e)) / 2e-6 for e in np.eye(3) * 1e-6], axis=1)
        S2 = Jfd @ Sc @ Jfd.T + cv.DILATION * np.eye(2)
        got = np.array([[P.cov2d[g, 0], P.cov2d[g, 1]], [P.cov2d[g, 1], P.cov2d[g, 2]]])
        assert np.allclose(got, S2, rtol=1e-6, atol=1e-9)
        assert np.allclose(P.conic[g], [np.linalg.inv(S2)[0, 0], np.linalg.inv(S2)[0, 1], np.linalg.inv(S2)[1, 1]], rtol=1e-6)
        assert np.allclose([P.u[g], P.v[g]], pi(pc), rtol=1e-12)
        assert abs(P.lam[g] - np.linalg.eigvalsh(got).max()) <= 1e-9 * P.lam[g]


def test_culls():
    cam = synth.identity_camera(64, 64)
    means = [[0, 0, 0.1], [0, 0, 3.0], [10.0, 0, 3.0], [0, 0, -2.0]]
    sc = stack_scene(means, [[-3] * 3] * 4, [[1, 0, 0, 0]] * 4, [0] * 4, [[.5] * 3] * 4)
    P = project(sc, cam)
    assert list(P.valid) == [False, True, False, False]
    assert list(P.touched > 0) == [False, True, False, False]


# ---------------------------------------------------------------- compositing

def test_single_gaussian_closed_form():
    cam = synth.identity_camera(64, 48)
    scene = one_gaussian_scene((0.05, -0.02, 3.0), [-2.3, -2.8, -2.5], [0.9, 0.1, -0.3, 0.2], 0.4, [0.2, 0.6, 0.9])
    fr = oracle.render_forward(scene, cam, bg=(0, 0, 0))
    P = fr.proj
    cov = np.array([[P.cov2d[0, 0], P.cov2d[0, 1]], [P.cov2d[0, 1], P.cov2d[0, 2]]])
    Q = np.linalg.inv(cov)
    o = 1 / (1 + math.exp(-float(np.float32(0.4))))
    c = P.rgb[0]
    x0, y0, x1, y1 = P.rect[0]
    img = fr.image
    for iy in range(48):
        for ix in range(64):
            inside = x0 <= ix // 16 <= x1 and y0 <= iy // 16 <= y1
            d = np.array([P.u[0] - (ix + 0.5), P.v[0] - (iy + 0.5)])
            ap = o * math.exp(-0.5 * d @ Q @ d)
            a = min(ap, cv.ALPHA_MAX)
            if not inside or a < cv.ALPHA_MIN:
                a, g = 0.0, np.zeros(2)
            else:
                g = a * (Q @ d) if ap < cv.ALPHA_MAX else np.zeros(2)
            assert np.allclose(img.rgb[:, iy, ix], c * a, atol=1e-13)
            assert abs(img.alpha[iy, ix] - a) < 1e-13
            assert abs(img.depth[iy, ix] - P.z[0] * a) < 1e-12
            assert np.allclose(img.dcdx[:, iy, ix], c * g[0], atol=1e-12)
            assert np.allclose(img.dcdy[:, iy, ix], c * g[1], atol=1e-12)


def test_two_gaussian_stack_closed_form_and_product_rule():
    cam = synth.identity_camera(32, 32)
    sc = stack_scene([[0.01, 0.0, 2.0], [-0.02, 0.01, 3.0]], [[-2.5] * 3, [-2.0] * 3],
                     [[1, 0, 0, 0], [0.8, 0.3, 0.1, -0.2]], [0.2, 1.0], [[1, 0, 0], [0, 0, 1]])
    fr = oracle.render_forward(sc, cam, bg=(0.1, 0.2, 0.3))
    P = fr.proj
    assert P.z[0] < P.z[1]
    ix, iy = 17, 14
    vals = []
    for g in range(2):
        cov = np.array([[P.cov2d[g, 0], P.cov2d[g, 1]], [P.cov2d[g, 1], P.cov2d[g, 2]]])
        Q = np.linalg.inv(cov)
        d = np.array([P.u[g] - (ix + 0.5), P.v[g] - (iy + 0.5)])
        a = P.opacity[g] * math.exp(-0.5 * d @ Q @ d)
        assert cv.ALPHA_MIN < a < cv.ALPHA_MAX
        vals.append((a, a * (Q @ d), P.rgb[g]))
    (a1, g1, c1), (a2, g2, c2) = vals
    bg = np.array([0.1, 0.2, 0.3])
    C = c1 * a1 + c2 * a2 * (1 - a1) + bg * (1 - a1) * (1 - a2)
    dTfinal = -g1 * (1 - a2) - (1 - a1) * g2
    dC = np.outer(g1, c1) + np.outer(g2 * (1 - a1) - a2 * g1, c2) + np.outer(dTfinal, bg)
    img = fr.image
    assert np.allclose(img.rgb[:, iy, ix], C, atol=1e-13)
    assert np.allclose(img.dcdx[:, iy, ix], dC[0], atol=1e-12)
    assert np.allclose(img.dcdy[:, iy, ix], dC[1], atol=1e-12)
    assert abs(img.alpha[iy, ix] - (1 - (1 - a1) * (1 - a2))) < 1e-13


@pytest.mark.parametrize("alpha", [0.5, 0.3, 0.9])
def test_identical_layers_stop_count(alpha):
    # n identical layers: blended count = min(n, max{k : (1-a)^k >= T_min})
    n = 40
    logit = math.log(alpha / (1 - alpha))
    means = [[0.0, 0.0, 2.0 + 0.01 * i] for i in range(n)]
    sc = stack_scene(means, [[-1.0] * 3] * n, [[1, 0, 0, 0]] * n, [logit] * n, [[0.5] * 3] * n)
    cam = synth.identity_camera(32, 32)
    fr = oracle.render_forward(sc, cam)
    a = float(fr.proj.opacity[0] * math.exp(-0.5 * ((fr.proj.u[0] - 16.5) ** 2 * fr.proj.conic[0, 0])))
    a_list = []
    P = fr.proj
    for g in range(n):
        d = np.array([P.u[g] - 16.5, P.v[g] - 16.5])
        Q = np.array([[P.conic[g, 0], P.conic[g, 1]], [P.conic[g, 1], P.conic[g, 2]]])
        a_list.append(P.opacity[g] * math.exp(-0.5 * d @ Q @ d))
    T, k = 1.0, 0
    while k < n and T * (1 - a_list[k]) >= cv.T_MIN:
        T *= 1 - a_list[k]
        k += 1
    assert fr.image.n_contrib[16, 16] == k == fr.image.blended[16, 16]
    expect = min(n, math.floor(math.log(cv.T_MIN) / math.log(1 - a)))
    assert abs(k - expect) <= 1
    assert abs(fr.image.final_T[16, 16] - T) < 1e-15


def test_telescoping_alpha_identity_on_random_scene():
    scene = synth.random_scene_small(7, 300, 1)
    cam = synth.identity_camera(48, 48)
    fr = oracle.render_forward(scene, cam)
    P = fr.proj
    lists = {}
    rng = np.random.default_rng(0)
    for _ in range(40):
        ix, iy = int(rng.integers(48)), int(rng.integers(48))
        tile = (iy // 16) * P.tiles_x + ix // 16
        lst = lists.setdefault(tile, brute.tile_list(P, tile))
        prod, n = 1.0, 0
        for k, g in enumerate(lst):
            d = np.array([P.u[g] - ix - 0.5, P.v[g] - iy - 0.5])
            Q = np.array([[P.conic[g, 0], P.conic[g, 1]], [P.conic[g, 1], P.conic[g, 2]]])
            a = min(P.opacity[g] * math.exp(-0.5 * d @ Q @ d), cv.ALPHA_MAX)
            if a < cv.ALPHA_MIN:
                continue
            if prod * (1 - a) < cv.T_MIN:
                break
            prod *= 1 - a
        assert abs(fr.image.alpha[iy, ix] - (1 - prod)) < 1e-12


def test_image_gradient_matches_finite_differences():
    scene = synth.random_scene_small(8, 200, 2)
    cam = synth.identity_camera(48, 32)
    bg = (0.2, 0.1, 0.4)
    fr = oracle.render_forward(scene, cam, bg=bg)
    rng = np.random.default_rng(1)
    h = 1e-5
    checked = 0
    for _ in range(60):
        ix, iy = int(rng.integers(48)), int(rng.integers(32))
        tile = (iy // 16) * fr.proj.tiles_x + ix // 16
        base = composite.composite_pixel(fr.proj, fr.values, fr.ranges, tile, ix, iy, bg)
        ok = True
        fd = []
        for e in ((h, 0), (0, h)):
            p = composite.composite_pixel(fr.proj, fr.values, fr.ranges, tile, ix, iy, bg,
                                          at=(ix + 0.5 + e[0], iy + 0.5 + e[1]))
            m = composite.composite_pixel(fr.proj, fr.values, fr.ranges, tile, ix, iy, bg,
                                          at=(ix + 0.5 - e[0], iy + 0.5 - e[1]))
            if p["n_contrib"] != base["n_contrib"] or m["n_contrib"] != base["n_contrib"]:
                ok = False
            fd.append((p["rgb"] - m["rgb"]) / (2 * h))
        if not ok or fr.image.ambiguous.get((ix, iy)):
            continue
        assert np.allclose(fd[0], fr.image.dcdx[:, iy, ix], atol=1e-6), (ix, iy)
        assert np.allclose(fd[1], fr.image.dcdy[:, iy, ix], atol=1e-6), (ix, iy)
        checked += 1
    assert checked > 40


# ---------------------------------------------------------------- binning + sort

def test_keys_sorted_stable_and_ranges_cover_all():
    scene, cam = synth.gen_cfg1(0, 2000, 64, 64)
    P = project(scene, cam)
    keys, vals = binning.emit_keys(P)
    sk, sv, rg = binning.bin_and_sort(P)
    assert np.all(sk[1:] >= sk[:-1])
    eq = sk[1:] == sk[:-1]
    assert np.all(sv[1:][eq] > sv[:-1][eq])
    assert sorted(zip(keys.tolist(), vals.tolist())) == list(zip(sk.tolist(), sv.tolist()))
    assert int((rg[:, 1] - rg[:, 0]).sum()) == sk.size == int(P.touched.sum())
    tiles = (sk >> np.uint64(32)).astype(np.int64)
    for t in range(rg.shape[0]):
        s, e = rg[t]
        assert np.all(tiles[s:e] == t)


def test_equal_depth_ties_break_by_index():
    n = 6
    means = [[0.001 * i, 0.0, 3.0] for i in range(n)][::-1]
    sc = stack_scene(means, [[-3] * 3] * n, [[1, 0, 0, 0]] * n, [0] * n, [[.5] * 3] * n)
    cam = synth.identity_camera(32, 32)
    P = project(sc, cam)
    assert len(set(P.zkey.tolist())) == 1
    _, sv, rg = binning.bin_and_sort(P)
    for t in range(rg.shape[0]):
        s, e = rg[t]
        assert list(sv[s:e]) == sorted(sv[s:e])


def test_tile_path_is_bit_identical_to_brute_force():
    scene = synth.random_scene_small(9, 150, 1)
    cam = synth.identity_camera(40, 36)     # ragged right and bottom tiles
    bg = (0.3, 0.0, 0.1)
    fr = oracle.render_forward(scene, cam, bg=bg)
    lists = {}
    for iy in range(0, 36, 3):
        for ix in range(0, 40, 3):
            b = brute.render_pixel(fr.proj, ix, iy, bg, lists=lists)
            assert np.array_equal(b["rgb"], fr.image.rgb[:, iy, ix])
            assert b["alpha"] == fr.image.alpha[iy, ix]
            assert b["depth"] == fr.image.depth[iy, ix]
            assert np.array_equal(b["dcdx"], fr.image.dcdx[:, iy, ix])
            assert np.array_equal(b["dcdy"], fr.image.dcdy[:, iy, ix])
            assert b["n_contrib"] == fr.image.n_contrib[iy, ix]


def test_untruncated_difference_is_bounded_by_three_sigma_cut():
    scene = synth.random_scene_small(10, 60, 0)
    cam = synth.identity_camera(32, 32)
    fr = oracle.render_forward(scene, cam)
    worst = 0.0
    for iy in range(0, 32, 4):
        for ix in range(0, 32, 4):
            u = brute.render_pixel(fr.proj, ix, iy, (0, 0, 0), untruncated=True)
            worst = max(worst, float(np.abs(u["alpha"] - fr.image.alpha[iy, ix])))
    assert worst < 0.2     # information: truncation changes alpha by a few percent at most


def test_config1_sizes():
    scene, cam = synth.gen_cfg1()
    P = project(scene, cam)
    K = int(P.touched.sum())
    assert 25_000 < K < 40_000
    assert (P.touched > 0).sum() == 10_000
