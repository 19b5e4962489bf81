"""Reverse-mode adjoint of the forward pass with respect to the Gaussian
parameters (means, log-scales, quaternions, opacity logits, SH), written as
plain FP64 adjoint code.

The discrete decisions of the forward pass (culls, tile rectangles, list
order, skips, the stop, the alpha clamp and the colour clamp at 0) are held
fixed: the derivative is the one-sided derivative of the function those
decisions select.  The loss may depend on the rendered rgb, alpha and depth;
gradients through the image-gradient buffers (second order) are not formed.

Compositing adjoint, per pixel with blended Gaussians i (Eq. 2):
  rgb = sum_i c_i a_i T_i + T_N bg,  alpha = 1 - T_N,  depth = sum_i z_i a_i T_i
  dL/dc_i = G_rgb a_i T_i,  dL/dz_i = G_depth a_i T_i
  dL/da_i = G_rgb . (c_i T_i - (S_i + bg T_N)/(1 - a_i))
            + G_depth (z_i T_i - Sz_i/(1 - a_i)) + G_alpha T_N/(1 - a_i)
with S_i, Sz_i the colour and depth blended behind i.  Below the clamp,
a = o exp(-q/2): dL/do = dL/da a/o, dL/dq = -a/2 dL/da, and q depends on the
2D mean and the conic.  The projection adjoint then chains through the conic
(inverse of the 2D covariance), the EWA product J R_wc Sigma R_wc^T J^T, the
Jacobian's dependence on the view-space mean, Sigma = M M^T with M = R(q)
diag(exp(log_scale)), the sigmoid, and the SH colour including its view
direction.
"""

from __future__ import annotations

import dataclasses

import numpy as np

from . import conventions as cv
from . import sh as shmod
from .composite import composite_tile


@dataclasses.dataclass
class Grads2D:
    du: np.ndarray
    dv: np.ndarray
    dconic: np.ndarray   # [N,3]
    dopacity: np.ndarray
    drgb: np.ndarray     # [N,3]
    dz: np.ndarray


@dataclasses.dataclass
class ParamGrads:
    means: np.ndarray
    log_scales: np.ndarray
    quats: np.ndarray
    opacity_logits: np.ndarray
    sh: np.ndarray


def composite_backward(frame, d_rgb, d_alpha=None, d_depth=None, tiles=None) -> Grads2D:
    proj = frame.proj
    N = proj.n
    W, H = frame.width, frame.height
    bg = frame.bg
    g2 = Grads2D(np.zeros(N), np.zeros(N), np.zeros((N, 3)), np.zeros(N), np.zeros((N, 3)), np.zeros(N))
    n_tiles = proj.tiles_x * proj.tiles_y
    for t in (range(n_tiles) if tiles is None else tiles):
        out = composite_tile(proj, frame.values, frame.ranges, t, W, H, bg, trace=True, track=False)
        X, Y = out.px, out.py
        GC = d_rgb[:, Y, X].T.astype(np.float64)                      # [P,3]
        GA = np.zeros(X.size) if d_alpha is None else d_alpha[Y, X].astype(np.float64)
        GD = np.zeros(X.size) if d_depth is None else d_depth[Y, X].astype(np.float64)
        TN = out.final_T
        S = np.zeros((X.size, 3))
        Sz = np.zeros(X.size)
        for st in reversed(out.trace):
            b, a, Tb, g = st["pix"], st["alpha"], st["T"], st["g"]
            c = proj.rgb[g]
            z = proj.z[g]
            w = a * Tb
            g2.drgb[g] += (GC[b] * w[:, None]).sum(axis=0)
            g2.dz[g] += (GD[b] * w).sum()
            inv = 1.0 / (1.0 - a)
            da = ((GC[b] * (c[None, :] * Tb[:, None] - (S[b] + bg[None, :] * TN[b][:, None]) * inv[:, None])).sum(axis=1)
                  + GD[b] * (z * Tb - Sz[b] * inv) + GA[b] * TN[b] * inv)
            S[b] += c[None, :] * w[:, None]
            Sz[b] += z * w
            m = st["unclamped"]
            if not m.any():
                continue
            da, a_u = da[m], a[m]
            dx, dy = st["dx"][m], st["dy"][m]
            A, B, Cc = proj.conic[g]
            g2.dopacity[g] += (da * a_u / proj.opacity[g]).sum()
            dq = -0.5 * a_u * da
            g2.dconic[g, 0] += (dq * dx * dx).sum()
            g2.dconic[g, 1] += (dq * 2.0 * dx * dy).sum()
            g2.dconic[g, 2] += (dq * dy * dy).sum()
            g2.du[g] += (dq * 2.0 * (A * dx + B * dy)).sum()
            g2.dv[g] += (dq * 2.0 * (B * dx + Cc * dy)).sum()
    return g2


def project_backward(scene, cam, proj, g2: Grads2D) -> ParamGrads:
    N = proj.n
    live = proj.touched > 0
    R = np.asarray(cam.R_wc, dtype=np.float64)
    fx, fy = float(cam.fx), float(cam.fy)

    # opacity: o = sigmoid(l)
    d_logit = g2.dopacity * proj.opacity * (1.0 - proj.opacity)

    # colour: rgb = max(sum_k sh_k Y_k(d) + 0.5, 0), d = (mean - centre)/|mean - centre|
    drr = g2.drgb * (proj.rgb_raw > 0.0)
    Y = shmod.basis(proj.dirs, scene.sh_degree)
    dY = shmod.basis_grad(proj.dirs, scene.sh_degree)           # [N,K,3]
    d_sh = Y[:, :, None] * drr[:, None, :]
    coeff = scene.sh.astype(np.float64)
    d_d = np.einsum("nc,nkc,nkj->nj", drr, coeff, dY)
    d_dir = (d_d - proj.dirs * (proj.dirs * d_d).sum(axis=1, keepdims=True)) / proj.dir_len[:, None]
    d_mean = d_dir.copy()

    # 2D mean: u = fx x/z + cx
    dgx = fx * g2.du
    dgy = fy * g2.dv

    # conic = inverse of (a, b, c)
    a, b, c = proj.cov2d[:, 0], proj.cov2d[:, 1], proj.cov2d[:, 2]
    det = np.where(proj.det > 0.0, proj.det, 1.0)
    d2 = det * det
    dA, dB, dC = g2.dconic[:, 0], g2.dconic[:, 1], g2.dconic[:, 2]
    da = dA * (-c * c / d2) + dB * (b * c / d2) + dC * (-b * b / d2)
    db = dA * (2.0 * b * c / d2) + dB * (-1.0 / det - 2.0 * b * b / d2) + dC * (2.0 * a * b / d2)
    dc = dA * (-b * b / d2) + dB * (a * b / d2) + dC * (-a * a / d2)

    # Sigma' = Tm Sigma Tm^T (+ dilation on the diagonal)
    Tm, Sig = proj.Tm, proj.cov3d
    T0, T1 = Tm[:, 0, :], Tm[:, 1, :]
    ST0 = np.einsum("nkl,nl->nk", Sig, T0)
    ST1 = np.einsum("nkl,nl->nk", Sig, T1)
    dSig = (da[:, None, None] * T0[:, :, None] * T0[:, None, :]
            + db[:, None, None] * T0[:, :, None] * T1[:, None, :]
            + dc[:, None, None] * T1[:, :, None] * T1[:, None, :])
    dT0 = 2.0 * da[:, None] * ST0 + db[:, None] * ST1
    dT1 = 2.0 * dc[:, None] * ST1 + db[:, None] * ST0

    # Tm = J R_wc
    dJ0 = np.einsum("nk,lk->nl", dT0, R)
    dJ1 = np.einsum("nk,lk->nl", dT1, R)
    zs = np.where(proj.valid, proj.z, 1.0)
    j00, j11 = fx / zs, fy / zs
    dj00 = dJ0[:, 0] - dJ0[:, 2] * proj.gx
    dj11 = dJ1[:, 1] - dJ1[:, 2] * proj.gy
    dgx = dgx - dJ0[:, 2] * j00
    dgy = dgy - dJ1[:, 2] * j11
    dzv = g2.dz - dj00 * fx / (zs * zs) - dj11 * fy / (zs * zs)
    dxv = dgx / zs
    dyv = dgy / zs
    dzv = dzv - dgx * proj.x / (zs * zs) - dgy * proj.y / (zs * zs)
    dp = np.stack([dxv, dyv, dzv], axis=1)
    d_mean += dp @ R                                              # R^T dp

    # Sigma = M M^T, M = R(q) diag(s)
    rot, s = proj.rot, proj.scale
    M = rot * s[:, None, :]
    dM = np.einsum("nij,njk->nik", dSig + np.transpose(dSig, (0, 2, 1)), M)
    dR = dM * s[:, None, :]
    ds = (dM * rot).sum(axis=1)
    d_logs = ds * s

    # R(q) = I + s_q Q(q), s_q = 2/|q|^2
    q = scene.quats.astype(np.float64)
    w, x, y, z = q[:, 0], q[:, 1], q[:, 2], q[:, 3]
    n2 = np.where(proj.qnorm2 > 0.0, proj.qnorm2, 1.0)
    sq = 2.0 / n2
    Q = np.empty((N, 3, 3))
    Q[:, 0, 0] = -(y * y + z * z)
    Q[:, 0, 1] = x * y - w * z
    Q[:, 0, 2] = x * z + w * y
    Q[:, 1, 0] = x * y + w * z
    Q[:, 1, 1] = -(x * x + z * z)
    Q[:, 1, 2] = y * z - w * x
    Q[:, 2, 0] = x * z - w * y
    Q[:, 2, 1] = y * z + w * x
    Q[:, 2, 2] = -(x * x + y * y)
    zero = np.zeros(N)
    dQ = {
        "w": [[zero, -z, y], [z, zero, -x], [-y, x, zero]],
        "x": [[zero, y, z], [y, -2 * x, -w], [z, w, -2 * x]],
        "y": [[-2 * y, x, w], [x, zero, z], [-w, z, -2 * y]],
        "z": [[-2 * z, -w, x], [w, -2 * z, y], [x, y, zero]],
    }
    dRQ = (dR * Q).sum(axis=(1, 2))
    d_q = np.zeros((N, 4))
    for col, (name, comp) in enumerate(zip("wxyz", (w, x, y, z))):
        dsq = -2.0 * sq * comp / n2                               # d(2/n)/dq_k = -4 q_k / n^2
        acc = dsq * dRQ
        for i in range(3):
            for j in range(3):
                acc = acc + sq * dR[:, i, j] * dQ[name][i][j]
        d_q[:, col] = acc

    mask = live.astype(np.float64)
    return ParamGrads(means=d_mean * mask[:, None], log_scales=d_logs * mask[:, None],
                      quats=d_q * mask[:, None], opacity_logits=d_logit * mask,
                      sh=d_sh * mask[:, None, None])


def backward(scene, cam, frame, d_rgb, d_alpha=None, d_depth=None):
    g2 = composite_backward(frame, d_rgb, d_alpha, d_depth)
    return project_backward(scene, cam, frame.proj, g2), g2


def l2_loss_and_grad(frame_image_rgb, target):
    """L = sum over pixels and channels of (rgb - target)^2, dL/drgb = 2 (rgb - target)."""
    diff = frame_image_rgb - target
    return float((diff * diff).sum()), 2.0 * diff
