"""Per-Gaussian projection: Eq. 1 primitives with Sigma = R S S^T R^T,
EWA splatting to a 2D Gaussian, 3-sigma screen radius and tile rectangle,
SH colour and opacity (Sec. 3).

Every geometric quantity that decides a sort key or a tile rectangle (view
z, the 2D mean u, v, the 2D covariance, its largest eigenvalue, the radius and
the rectangle) is computed in FP64 as explicit scalar operations in a fixed
order, each a correctly rounded IEEE operation: no matrix products (they
reassociate) and no fused multiply-add.  NumPy evaluates ``a*b + c`` as two
rounded operations, which is the order written here.
"""

from __future__ import annotations

import dataclasses

import numpy as np

from . import conventions as cv
from . import sh as shmod


@dataclasses.dataclass
class Projected:
    n: int
    valid: np.ndarray        # bool: passed near / guard / degeneracy culls
    x: np.ndarray            # view-space position (FP64)
    y: np.ndarray
    z: np.ndarray
    gx: np.ndarray           # x/z, y/z
    gy: np.ndarray
    u: np.ndarray            # 2D mean in pixels (FP64)
    v: np.ndarray
    cov2d: np.ndarray        # [N,3] (a, b, c) dilated 2D covariance
    det: np.ndarray
    conic: np.ndarray        # [N,3] (A, B, C) inverse of the 2D covariance
    lam: np.ndarray          # largest eigenvalue
    radius: np.ndarray       # integer-valued FP64
    rect: np.ndarray         # [N,4] int64 (tx0, ty0, tx1, ty1), inclusive
    touched: np.ndarray      # int64 tiles covered (0 when culled or off-screen)
    opacity: np.ndarray
    rgb: np.ndarray          # [N,3] clamped colour
    rgb_raw: np.ndarray      # [N,3] before the clamp at 0
    dirs: np.ndarray         # [N,3] unit view directions (mean - camera centre)
    dir_len: np.ndarray
    rot: np.ndarray          # [N,3,3] R(q)
    normal: np.ndarray       # [N,3] unit surface normal in camera axes, facing the camera
    scale: np.ndarray        # [N,3] exp(log_scale)
    cov3d: np.ndarray        # [N,3,3]
    J: np.ndarray            # [N,2,3]
    Tm: np.ndarray           # [N,2,3] J R_wc
    qnorm2: np.ndarray
    tiles_x: int
    tiles_y: int

    @property
    def zkey(self) -> np.ndarray:
        """float32 bit pattern of view z (positive, so it orders like uint)."""
        return self.z.astype(np.float32).view(np.uint32)


def quat_to_rot(q: np.ndarray):
    """Rotation from a not necessarily unit quaternion (w, x, y, z):
    R = I + s Q(q) with s = 2 / |q|^2 (no square root)."""
    w, x, y, z = (q[:, i].astype(np.float64) for i in range(4))
    n = ((w * w + x * x) + y * y) + z * z
    s = np.where(n > 0.0, 2.0 / np.where(n > 0.0, n, 1.0), 0.0)
    R = np.empty((q.shape[0], 3, 3))
    R[:, 0, 0] = 1.0 - s * (y * y + z * z)
    R[:, 0, 1] = s * (x * y - w * z)
    R[:, 0, 2] = s * (x * z + w * y)
    R[:, 1, 0] = s * (x * y + w * z)
    R[:, 1, 1] = 1.0 - s * (x * x + z * z)
    R[:, 1, 2] = s * (y * z - w * x)
    R[:, 2, 0] = s * (x * z - w * y)
    R[:, 2, 1] = s * (y * z + w * x)
    R[:, 2, 2] = 1.0 - s * (x * x + y * y)
    return R, n


def camera_centre(cam) -> np.ndarray:
    """c = -R_wc^T t, each component ((R0k t0 + R1k t1) + R2k t2) negated."""
    R, t = cam.R_wc, cam.t
    return np.array([-((R[0, k] * t[0] + R[1, k] * t[1]) + R[2, k] * t[2]) for k in range(3)])


def project(scene, cam, near: float = cv.NEAR, dilation: float = cv.DILATION) -> Projected:
    n = scene.n
    R = np.asarray(cam.R_wc, dtype=np.float64)
    t = np.asarray(cam.t, dtype=np.float64)
    W, H = int(cam.width), int(cam.height)
    fx, fy, cx, cy = float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy)
    TX = (W + cv.TILE - 1) // cv.TILE
    TY = (H + cv.TILE - 1) // cv.TILE

    mx = scene.means[:, 0].astype(np.float64)
    my = scene.means[:, 1].astype(np.float64)
    mz = scene.means[:, 2].astype(np.float64)

    # view-space position, pinned order ((r0 mx + r1 my) + r2 mz) + t
    x = ((R[0, 0] * mx + R[0, 1] * my) + R[0, 2] * mz) + t[0]
    y = ((R[1, 0] * mx + R[1, 1] * my) + R[1, 2] * mz) + t[1]
    z = ((R[2, 0] * mx + R[2, 1] * my) + R[2, 2] * mz) + t[2]

    valid = z >= near
    zs = np.where(valid, z, 1.0)
    gx = x / zs
    gy = y / zs
    limx = cv.GUARD * ((0.5 * W) / fx)
    limy = cv.GUARD * ((0.5 * H) / fy)
    valid &= ~((gx < -limx) | (gx > limx) | (gy < -limy) | (gy > limy))

    # Sigma = R S S^T R^T (Sec. 3), S = diag(exp(log_scale))
    rot, qn = quat_to_rot(scene.quats)
    valid &= qn > 0.0
    scale = np.exp(scene.log_scales.astype(np.float64))
    M = rot * scale[:, None, :]                     # M_ij = R_ij s_j
    cov3d = np.empty((n, 3, 3))
    for i in range(3):
        for j in range(3):
            cov3d[:, i, j] = (M[:, i, 0] * M[:, j, 0] + M[:, i, 1] * M[:, j, 1]) + M[:, i, 2] * M[:, j, 2]

    # EWA: local affine approximation J of the perspective map at the mean
    j00 = fx / zs
    j11 = fy / zs
    j02 = -(j00 * gx)
    j12 = -(j11 * gy)
    J = np.zeros((n, 2, 3))
    J[:, 0, 0] = j00
    J[:, 0, 2] = j02
    J[:, 1, 1] = j11
    J[:, 1, 2] = j12
    Tm = np.empty((n, 2, 3))
    for k in range(3):
        Tm[:, 0, k] = j00 * R[0, k] + j02 * R[2, k]
        Tm[:, 1, k] = j11 * R[1, k] + j12 * R[2, k]
    # U = Tm Sigma, then Sigma' = U Tm^T
    U = np.empty((n, 2, 3))
    for i in range(2):
        for k in range(3):
            U[:, i, k] = (Tm[:, i, 0] * cov3d[:, 0, k] + Tm[:, i, 1] * cov3d[:, 1, k]) + Tm[:, i, 2] * cov3d[:, 2, k]

    def quad(i, j):
        return (U[:, i, 0] * Tm[:, j, 0] + U[:, i, 1] * Tm[:, j, 1]) + U[:, i, 2] * Tm[:, j, 2]

    a = quad(0, 0) + dilation
    b = quad(0, 1)
    c = quad(1, 1) + dilation
    det = a * c - b * b
    valid &= det > 0.0
    dets = np.where(det > 0.0, det, 1.0)
    conic = np.stack([c / dets, -b / dets, a / dets], axis=1)

    mid = 0.5 * (a + c)
    lam = mid + np.sqrt(np.maximum(0.0, mid * mid - det))
    radius = np.ceil(cv.SIGMA_CUT * np.sqrt(np.maximum(lam, 0.0)))

    u = fx * gx + cx
    v = fy * gy + cy

    tx0 = np.maximum(np.floor((u - radius) / cv.TILE), 0.0)
    tx1 = np.minimum(np.floor((u + radius) / cv.TILE), float(TX - 1))
    ty0 = np.maximum(np.floor((v - radius) / cv.TILE), 0.0)
    ty1 = np.minimum(np.floor((v + radius) / cv.TILE), float(TY - 1))
    nonempty = valid & (tx0 <= tx1) & (ty0 <= ty1)
    rect = np.zeros((n, 4), dtype=np.int64)
    rect[nonempty, 0] = tx0[nonempty].astype(np.int64)
    rect[nonempty, 1] = ty0[nonempty].astype(np.int64)
    rect[nonempty, 2] = tx1[nonempty].astype(np.int64)
    rect[nonempty, 3] = ty1[nonempty].astype(np.int64)
    touched = np.where(nonempty, (rect[:, 2] - rect[:, 0] + 1) * (rect[:, 3] - rect[:, 1] + 1), 0)

    # colour: one view direction per Gaussian (mean minus camera centre)
    cc = camera_centre(cam)
    dvec = np.stack([mx - cc[0], my - cc[1], mz - cc[2]], axis=1)
    dlen = np.sqrt((dvec[:, 0] * dvec[:, 0] + dvec[:, 1] * dvec[:, 1]) + dvec[:, 2] * dvec[:, 2])
    dirs = dvec / np.where(dlen > 0.0, dlen, 1.0)[:, None]
    Y = shmod.basis(dirs, scene.sh_degree)                   # [N,K]
    coeff = scene.sh.astype(np.float64)                      # [N,K,3]
    rgb_raw = np.einsum("nk,nkc->nc", Y, coeff) + cv.COLOR_OFFSET
    rgb = np.maximum(rgb_raw, 0.0)

    opacity = 1.0 / (1.0 + np.exp(-scene.opacity_logits.astype(np.float64)))

    # surface normal (the normal maps N and Nv of Sec. 4.1 and 4.2, rendered
    # the RaDe-GS way, Sec. 5.1): the direction of the ellipsoid's shortest
    # axis, i.e. the column of R(q) whose scale is smallest (the first one on
    # ties, compared on the float32 log-scales), in camera axes
    # ((Rc_i0 n0 + Rc_i1 n1) + Rc_i2 n2), and flipped where it points away
    # from the camera (((n0 x + n1 y) + n2 z) > 0, (x, y, z) the view-space mean)
    kmin = np.argmin(scene.log_scales, axis=1)
    nw = rot[np.arange(n), :, kmin]
    ncam = np.stack([(R[i, 0] * nw[:, 0] + R[i, 1] * nw[:, 1]) + R[i, 2] * nw[:, 2] for i in range(3)], axis=1)
    away = ((ncam[:, 0] * x + ncam[:, 1] * y) + ncam[:, 2] * z) > 0.0
    normal = np.where(away[:, None], -ncam, ncam)

    return Projected(n=n, valid=valid, x=x, y=y, z=z, gx=gx, gy=gy, u=u, v=v,
                     cov2d=np.stack([a, b, c], axis=1), det=det, conic=conic, lam=lam,
                     radius=radius, rect=rect, touched=touched.astype(np.int64),
                     opacity=opacity, rgb=rgb, rgb_raw=rgb_raw, dirs=dirs, dir_len=dlen,
                     rot=rot, normal=normal, scale=scale, cov3d=cov3d, J=J, Tm=Tm, qnorm2=qn,
                     tiles_x=TX, tiles_y=TY)
