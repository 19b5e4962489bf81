"""Gradient-aware interpolation of a low-resolution image to S times its size
in each axis (3DGS^3 Sec. 4.1, Eq. 5-7), with a fixed least-squares matrix.

TEST INFRASTRUCTURE ONLY (see the package docstring): nothing in the product
imports this module.  FP64 NumPy throughout.

Eq. 5 asks a bivariate polynomial f to match, at the 3x3 block of pixel
centres around pixel (x0, y0), the image values and both first derivatives:
27 conditions.  Eq. 6 pairs that block with the S x S block of
high-resolution pixels covering (x0, y0), and Eq. 7 writes each of those as
one linear combination of the 27 inputs: Vec(I_hat) = M [Vec(I); Vec(I_x);
Vec(I_y)].  The paper learns M inside a Conv/TConv pair; the readings here
make it fixed:
  * f ranges over the polynomials of total degree <= 5, x^a y^b with
    a + b <= 5 (21 terms); 27 conditions over-determine them, so f is their
    least-squares fit with equal weights, and M = E pinv(A), where A
    (27 x 21, full column rank) holds the basis values and derivatives at
    the 9 nodes and E (S^2 x 21) the basis values at the S^2
    high-resolution pixel centres.  (The bicubic space would not do: the
    bicubic (x^3 - x)(y^3 - y) vanishes with its gradient at all 9 nodes, so
    its 16 x 27 system has rank 15.)
  * coordinates are in low-resolution pixel units relative to the centre of
    (x0, y0); node (i, j), i, j in {-1, 0, 1}, sits at offset (i, j); the
    high-resolution pixel (k, l), k, l in 0..S-1, of the block sits at
    ((k + 0.5)/S - 0.5, (l + 0.5)/S - 0.5);
  * the 27 inputs are ordered values, then x-derivatives, then
    y-derivatives, each over the nodes with n = 3 (j + 1) + (i + 1);
  * nodes outside the image take the nearest edge pixel's value and
    derivatives (clamp to edge);
  * derivatives are per low-resolution pixel, as the rasterizer's dC/dx.
Any polynomial of total degree <= 5 sampled with its exact derivatives is
reproduced exactly, which is what pins this oracle.
"""

from __future__ import annotations

import numpy as np

NODES = [(i, j) for j in (-1, 0, 1) for i in (-1, 0, 1)]   # n = 3 (j + 1) + (i + 1)
POWERS = [(a, b) for b in range(6) for a in range(6) if a + b <= 5]   # x^a y^b, 21 terms


def _basis(x: float, y: float) -> np.ndarray:
    return np.array([x ** a * y ** b for a, b in POWERS], dtype=np.float64)


def _basis_dx(x: float, y: float) -> np.ndarray:
    return np.array([a * x ** (a - 1) * y ** b if a else 0.0 for a, b in POWERS], dtype=np.float64)


def _basis_dy(x: float, y: float) -> np.ndarray:
    return np.array([b * x ** a * y ** (b - 1) if b else 0.0 for a, b in POWERS], dtype=np.float64)


def sub_offsets(S: int):
    """Offsets (dx, dy) of the S x S high-resolution pixel centres, row-major (l, k)."""
    c = (np.arange(S) + 0.5) / S - 0.5
    return [(c[k], c[l]) for l in range(S) for k in range(S)]


def constraint_matrix() -> np.ndarray:
    A = np.zeros((27, len(POWERS)))
    for n, (i, j) in enumerate(NODES):
        A[n] = _basis(i, j)
        A[9 + n] = _basis_dx(i, j)
        A[18 + n] = _basis_dy(i, j)
    return A


def matrix_M(S: int) -> np.ndarray:
    """M (S^2 x 27): row s = high-resolution pixel (k, l) with s = l S + k."""
    E = np.stack([_basis(dx, dy) for dx, dy in sub_offsets(S)])
    return E @ np.linalg.pinv(constraint_matrix())


def gather(img: np.ndarray, gx: np.ndarray, gy: np.ndarray, x0: int, y0: int) -> np.ndarray:
    """The 27-vector of inputs of pixel (x0, y0) of one channel ([H, W] arrays)."""
    H, W = img.shape
    v = np.empty(27)
    for n, (i, j) in enumerate(NODES):
        x = min(max(x0 + i, 0), W - 1)
        y = min(max(y0 + j, 0), H - 1)
        v[n], v[9 + n], v[18 + n] = img[y, x], gx[y, x], gy[y, x]
    return v


def upsample(rgb: np.ndarray, dcdx: np.ndarray, dcdy: np.ndarray, S: int) -> np.ndarray:
    """rgb, dcdx, dcdy: [C, H, W]; returns [C, H S, W S]."""
    rgb, dcdx, dcdy = (np.asarray(a, dtype=np.float64) for a in (rgb, dcdx, dcdy))
    Cn, H, W = rgb.shape
    M = matrix_M(S)
    out = np.empty((Cn, H * S, W * S))
    for c in range(Cn):
        # all pixels at once: [H, W, 27] inputs
        V = np.empty((H, W, 27))
        ys, xs = np.arange(H), np.arange(W)
        for n, (i, j) in enumerate(NODES):
            yy = np.clip(ys + j, 0, H - 1)[:, None]
            xx = np.clip(xs + i, 0, W - 1)[None, :]
            V[:, :, n] = rgb[c][yy, xx]
            V[:, :, 9 + n] = dcdx[c][yy, xx]
            V[:, :, 18 + n] = dcdy[c][yy, xx]
        blk = V @ M.T                                    # [H, W, S*S], s = l S + k
        out[c] = blk.reshape(H, W, S, S).transpose(0, 2, 1, 3).reshape(H * S, W * S)
    return out
