"""Gradient-aware interpolation (Sec. 4.1, Eq. 5-7) on the GPU through the C
ABI against the FP64 oracle: every output at S = 1..4 on ragged rasters,
the full 960x540 -> 3840x2160 case, polynomial reproduction, edge rasters."""

import numpy as np
import pytest

import synth
from oracle import upsample as U

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2605_11489_amd import render as R  # noqa: E402

# FP32 sums of 27 products with |M| < 2 of inputs of order 1
TOL = 2e-5


def say(msg):
    print(msg, flush=True)


def run(img, gx, gy, S):
    t = [torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda() for a in (img, gx, gy)]
    out = R.gradient_upsample(*t, S)
    torch.cuda.synchronize()
    return out.cpu().numpy().astype(np.float64)


@pytest.mark.parametrize("S", [1, 2, 3, 4])
def test_matches_oracle_ragged(S):
    say(f"case: upsample 100x70 S={S} seed 5")
    img, gx, gy = synth.image_fields(5, 100, 70)
    g = run(img, gx, gy, S)
    ref = U.upsample(img, gx, gy, S)
    err = np.abs(g - ref).max()
    say(f"  max abs err {err:.3g}")
    assert err < TOL


@pytest.mark.parametrize("W,H", [(1, 1), (17, 1), (1, 23), (16, 16)])
def test_edge_rasters(W, H):
    say(f"case: upsample {W}x{H} S=4")
    img, gx, gy = synth.image_fields(6, W, H)
    assert np.abs(run(img, gx, gy, 4) - U.upsample(img, gx, gy, 4)).max() < TOL


def test_full_size_960x540_scale4():
    say("case: upsample 960x540 -> 3840x2160 seed 7")
    img, gx, gy = synth.image_fields(7, 960, 540)
    g = run(img, gx, gy, 4)
    ref = U.upsample(img, gx, gy, 4)
    err = np.abs(g - ref).max()
    say(f"  max abs err {err:.3g}")
    assert err < TOL


def test_quintic_reproduced_on_gpu():
    say("case: degree-5 polynomial 40x30 S=4")
    rng = np.random.default_rng(8)
    coef = {(a, b): rng.normal() * 0.5 for a in range(6) for b in range(6) if a + b <= 5}
    W, H, sc = 40, 30, 0.05
    xs, ys = (np.arange(W) + 0.5) * sc, (np.arange(H) + 0.5) * sc
    X, Y = np.meshgrid(xs, ys)
    I = sum(c * X ** a * Y ** b for (a, b), c in coef.items())
    Ix = sum(c * a * X ** (a - 1) * Y ** b * sc for (a, b), c in coef.items() if a)
    Iy = sum(c * b * X ** a * Y ** (b - 1) * sc for (a, b), c in coef.items() if b)
    g = run(np.stack([I] * 3), np.stack([Ix] * 3), np.stack([Iy] * 3), 4)[0]
    Xh, Yh = np.meshgrid((np.arange(W * 4) + 0.5) / 4 * sc, (np.arange(H * 4) + 0.5) / 4 * sc)
    ref = sum(c * Xh ** a * Yh ** b for (a, b), c in coef.items())
    inner = (slice(4, (H - 1) * 4), slice(4, (W - 1) * 4))
    assert np.abs(g[inner] - ref[inner]).max() < 1e-4 * max(1.0, np.abs(ref).max())
