"""Real spherical harmonics up to degree 3 (view-dependent colour, Sec. 3,
Eq. 2: c_i is predicted from SH coefficients).

Reading: the real orthonormal basis with the Condon-Shortley phase, ordered
m = -l..l within each degree l (the ordering used by 3DGS coefficient files).
Every constant is computed here from its closed form
sqrt((2l+1)/(4 pi) (l-|m|)!/(l+|m|)!) times the polynomial normalisation, so
a reader can check each line against a table of real SH.
"""

import math

import numpy as np

PI = math.pi
C0 = 1.0 / (2.0 * math.sqrt(PI))
C1 = math.sqrt(3.0 / (4.0 * PI))
C2A = math.sqrt(15.0 / (4.0 * PI))
C2B = math.sqrt(5.0 / (16.0 * PI))
C2C = math.sqrt(15.0 / (16.0 * PI))
C3A = math.sqrt(35.0 / (32.0 * PI))
C3B = math.sqrt(105.0 / (4.0 * PI))
C3C = math.sqrt(21.0 / (32.0 * PI))
C3D = math.sqrt(7.0 / (16.0 * PI))
C3E = math.sqrt(105.0 / (16.0 * PI))


def basis(d: np.ndarray, degree: int) -> np.ndarray:
    """Y[..., k] for unit directions d[..., 3]; k = 0..(degree+1)^2-1."""
    x, y, z = d[..., 0], d[..., 1], d[..., 2]
    out = [np.full_like(x, C0)]
    if degree >= 1:
        out += [-C1 * y, C1 * z, -C1 * x]
    if degree >= 2:
        out += [C2A * x * y,
                -C2A * y * z,
                C2B * (2.0 * z * z - x * x - y * y),
                -C2A * x * z,
                C2C * (x * x - y * y)]
    if degree >= 3:
        out += [-C3A * y * (3.0 * x * x - y * y),
                C3B * x * y * z,
                -C3C * y * (4.0 * z * z - x * x - y * y),
                C3D * z * (2.0 * z * z - 3.0 * x * x - 3.0 * y * y),
                -C3C * x * (4.0 * z * z - x * x - y * y),
                C3E * z * (x * x - y * y),
                -C3A * x * (x * x - 3.0 * y * y)]
    return np.stack(out, axis=-1)


def basis_grad(d: np.ndarray, degree: int) -> np.ndarray:
    """dY_k/d(x,y,z) with x, y, z treated as independent: [..., K, 3]."""
    x, y, z = d[..., 0], d[..., 1], d[..., 2]
    zero = np.zeros_like(x)
    rows = [(zero, zero, zero)]
    if degree >= 1:
        rows += [(zero, -C1 + zero, zero),
                 (zero, zero, C1 + zero),
                 (-C1 + zero, zero, zero)]
    if degree >= 2:
        rows += [(C2A * y, C2A * x, zero),
                 (zero, -C2A * z, -C2A * y),
                 (-2.0 * C2B * x, -2.0 * C2B * y, 4.0 * C2B * z),
                 (-C2A * z, zero, -C2A * x),
                 (2.0 * C2C * x, -2.0 * C2C * y, zero)]
    if degree >= 3:
        rows += [(-C3A * 6.0 * x * y, -C3A * (3.0 * x * x - 3.0 * y * y), zero),
                 (C3B * y * z, C3B * x * z, C3B * x * y),
                 (C3C * 2.0 * x * y, -C3C * (4.0 * z * z - x * x - 3.0 * y * y), -C3C * 8.0 * y * z),
                 (-C3D * 6.0 * x * z, -C3D * 6.0 * y * z, C3D * (6.0 * z * z - 3.0 * x * x - 3.0 * y * y)),
                 (-C3C * (4.0 * z * z - 3.0 * x * x - y * y), C3C * 2.0 * x * y, -C3C * 8.0 * x * z),
                 (C3E * 2.0 * x * z, -C3E * 2.0 * y * z, C3E * (x * x - y * y)),
                 (-C3A * (3.0 * x * x - 3.0 * y * y), C3A * 6.0 * x * y, zero)]
    return np.stack([np.stack(r, axis=-1) for r in rows], axis=-2)
