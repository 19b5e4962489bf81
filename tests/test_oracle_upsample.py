"""Pins of the gradient-aware interpolation oracle (Sec. 4.1, Eq. 5-7) against
what the mathematics fixes: exact reproduction of polynomials of total degree
<= 5 sampled with their exact derivatives, the failure to reproduce a degree-6
term (so the
pins can tell), constants at the clamped border, and a brute-force per-pixel
evaluation of the least-squares fit."""

import numpy as np
import pytest

from oracle import upsample as U


def poly_image(coef, W, H, scale=0.2):
    """I(x, y) = sum c_ab X^a Y^b at pixel centres, X = scale (x + 0.5),
    with derivatives per pixel."""
    xs = (np.arange(W) + 0.5) * scale
    ys = (np.arange(H) + 0.5) * scale
    X, Y = np.meshgrid(xs, ys)
    I = np.zeros((H, W)); Ix = np.zeros((H, W)); Iy = np.zeros((H, W))
    for (a, b), c in coef.items():
        I += c * X ** a * Y ** b
        if a:
            Ix += c * a * X ** (a - 1) * Y ** b * scale
        if b:
            Iy += c * b * X ** a * Y ** (b - 1) * scale
    return I, Ix, Iy


def poly_at(coef, X, Y):
    return sum(c * X ** a * Y ** b for (a, b), c in coef.items())


@pytest.mark.parametrize("S", [1, 2, 3, 4])
def test_quintic_reproduced_exactly(S):
    rng = np.random.default_rng(S)
    coef = {(a, b): rng.normal() for a in range(6) for b in range(6) if a + b <= 5}
    W, H, scale = 11, 9, 0.2
    I, Ix, Iy = poly_image(coef, W, H, scale)
    out = U.upsample(I[None], Ix[None], Iy[None], S)[0]
    Xh = (np.arange(W * S) + 0.5) / S * scale
    Yh = (np.arange(H * S) + 0.5) / S * scale
    Xg, Yg = np.meshgrid(Xh, Yh)
    ref = poly_at(coef, Xg, Yg)
    inner = (slice(S, (H - 1) * S), slice(S, (W - 1) * S))   # away from the clamped border
    assert np.abs(out[inner] - ref[inner]).max() < 1e-9 * max(1.0, np.abs(ref).max())


def test_degree_six_not_reproduced():
    coef = {(6, 0): 1.0}
    W, H, scale = 9, 9, 0.5
    I, Ix, Iy = poly_image(coef, W, H, scale)
    out = U.upsample(I[None], Ix[None], Iy[None], 4)[0]
    Xh = (np.arange(W * 4) + 0.5) / 4 * scale
    ref = np.broadcast_to(Xh ** 6, out.shape)
    inner = (slice(4, 32), slice(4, 32))
    assert np.abs(out[inner] - ref[inner]).max() > 1e-4


def test_constant_everywhere_including_border():
    I = np.full((3, 5, 7), 0.37)
    Z = np.zeros_like(I)
    out = U.upsample(I, Z, Z, 4)
    assert np.abs(out - 0.37).max() < 1e-12


def test_matches_per_pixel_least_squares():
    """Brute force: solve the 27-condition least-squares problem of one pixel
    directly (lstsq) and evaluate the fitted polynomial at the sub-pixels."""
    rng = np.random.default_rng(4)
    I, Ix, Iy = rng.random((3, 6, 5))
    S = 3
    out = U.upsample(I[None], Ix[None], Iy[None], S)[0]
    for (x0, y0) in [(0, 0), (2, 3), (4, 5), (1, 2)]:
        v = U.gather(I, Ix, Iy, x0, y0)
        A = U.constraint_matrix()
        c, *_ = np.linalg.lstsq(A, v, rcond=None)
        for l in range(S):
            for k in range(S):
                dx, dy = (k + 0.5) / S - 0.5, (l + 0.5) / S - 0.5
                f = sum(cc * dx ** a * dy ** b for cc, (a, b) in zip(c, U.POWERS))
                assert abs(out[y0 * S + l, x0 * S + k] - f) < 1e-12


def test_value_weights_sum_to_one():
    for S in (1, 2, 4):
        M = U.matrix_M(S)
        assert np.allclose(M[:, :9].sum(1), 1.0, atol=1e-12)
