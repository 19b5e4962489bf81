"""Pin of the oracle's FP64 adjoint: central finite differences of the oracle's
own forward pass (h = 1e-4), excluding parameters whose +-h perturbation
changes any discrete decision of the forward pass.  CPU only."""

import numpy as np
import pytest

import oracle
import synth
from oracle import backward, composite


def decisions(frame):
    P = frame.proj
    sig = [P.rect.tobytes(), P.touched.tobytes(), (P.rgb_raw > 0).tobytes()]
    for t in range(P.tiles_x * P.tiles_y):
        out = composite.composite_tile(P, frame.values, frame.ranges, t, frame.width, frame.height,
                                       frame.bg, trace=True, track=False)
        for st in out.trace:
            sig.append((t, st["k"], st["g"], st["pix"].tobytes(), st["unclamped"].tobytes()))
    return sig


def loss(scene, cam, target, w_alpha, w_depth, bg):
    fr = oracle.render_forward(scene, cam, bg=bg, track=False)
    img = fr.image
    L = float(((img.rgb - target) ** 2).sum() + (w_alpha * img.alpha).sum() + (w_depth * img.depth).sum())
    return L, fr


FIELDS = ("means", "log_scales", "quats", "opacity_logits", "sh")


@pytest.mark.parametrize("seed,degree,bg", [(11, 3, (0.0, 0.0, 0.0)), (12, 1, (0.3, 0.5, 0.1))])
def test_backward_matches_central_differences(seed, degree, bg):
    scene = synth.random_scene_small(seed, 40, degree, lo=(-0.5, -0.5, 2.0), hi=(0.5, 0.5, 4.0),
                                     log_scale_mean=-2.6)
    cam = synth.look_at_camera((0.3, -0.2, -0.5), 32, 32, target=(0.0, 0.0, 3.0))
    rng = np.random.default_rng(seed)
    target = rng.uniform(0, 1, size=(3, 32, 32))
    w_alpha = rng.normal(size=(32, 32))
    w_depth = rng.normal(size=(32, 32)) * 0.1
    L0, fr = loss(scene, cam, target, w_alpha, w_depth, bg)
    sig0 = decisions(fr)
    d_rgb = 2.0 * (fr.image.rgb - target)
    pg, _ = backward.backward(scene, cam, fr, d_rgb, w_alpha, w_depth)
    h = 1e-4
    checked = skipped = 0
    worst = 0.0
    for field in FIELDS:
        arr = getattr(scene, field)
        flat = arr.reshape(-1)
        picks = rng.choice(flat.size, size=min(flat.size, 25), replace=False)
        for i in picks:
            vals = []
            flip = False
            for sgn in (1, -1):
                sc = scene.copy()
                a = getattr(sc, field).reshape(-1)
                a[i] = np.float32(np.float64(flat[i]) + sgn * h)
                Lp, frp = loss(sc, cam, target, w_alpha, w_depth, bg)
                if decisions(frp) != sig0:
                    flip = True
                    break
                vals.append((Lp, float(np.float64(a[i]) - np.float64(flat[i]))))
            if flip:
                skipped += 1
                continue
            (Lp, hp), (Lm, hm) = vals
            fd = (Lp - Lm) / (hp - hm)
            an = getattr(pg, field).reshape(-1)[i]
            err = abs(fd - an) / max(1.0, abs(an))
            worst = max(worst, err)
            assert err < 2e-3, (field, i, fd, an)
            checked += 1
    assert checked >= 60, (checked, skipped)


def test_backward_every_parameter_of_three_gaussians():
    """All 59 parameters (mean 3, log-scale 3, quaternion 4, opacity 1, SH 48)
    of the three Gaussians with the largest gradients, against central
    differences, so that a mistake confined to one component or coefficient
    index cannot hide between random picks."""
    seed, bg = 13, (0.2, 0.1, 0.4)
    scene = synth.random_scene_small(seed, 30, 3, lo=(-0.5, -0.5, 2.0), hi=(0.5, 0.5, 4.0), log_scale_mean=-2.4)
    cam = synth.look_at_camera((0.2, 0.1, -0.4), 28, 24, target=(0.0, 0.0, 3.0))
    rng = np.random.default_rng(seed)
    target = rng.uniform(0, 1, size=(3, 24, 28))
    w_alpha = rng.normal(size=(24, 28))
    w_depth = rng.normal(size=(24, 28)) * 0.1
    L0, fr = loss(scene, cam, target, w_alpha, w_depth, bg)
    sig0 = decisions(fr)
    pg, _ = backward.backward(scene, cam, fr, 2.0 * (fr.image.rgb - target), w_alpha, w_depth)
    mag = np.abs(pg.means).sum(axis=1)
    gs = np.argsort(-mag)[:3]
    h = 1e-4
    checked = 0
    for g in gs:
        for field in FIELDS:
            arr = getattr(scene, field)
            per = arr.reshape(arr.shape[0], -1).shape[1]
            for c in range(per):
                i = g * per + c
                vals = []
                flip = False
                for sgn in (1, -1):
                    sc = scene.copy()
                    a = getattr(sc, field).reshape(-1)
                    a[i] = np.float32(np.float64(arr.reshape(-1)[i]) + sgn * h)
                    Lp, frp = loss(sc, cam, target, w_alpha, w_depth, bg)
                    if decisions(frp) != sig0:
                        flip = True
                        break
                    vals.append((Lp, float(np.float64(a[i]) - np.float64(arr.reshape(-1)[i]))))
                if flip:
                    continue
                (Lp, hp), (Lm, hm) = vals
                fd = (Lp - Lm) / (hp - hm)
                an = getattr(pg, field).reshape(-1)[i]
                assert abs(fd - an) <= 2e-3 * max(1.0, abs(an)), (g, field, c, fd, an)
                checked += 1
    assert checked >= 150, checked
