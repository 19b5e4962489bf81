"""Pose-derived motion vectors and forward warping of the rasterizer's outputs
to another camera (3DGS^3 Sec. 4.2, Eq. 12 and Eq. 13).

TEST INFRASTRUCTURE ONLY (see the package docstring).  FP64 NumPy.

Eq. 12: for a pixel x of the source frame, V[x] = Proj(UnProj(x, P_src),
P_dst) - x.  Readings:
  * x is the pixel centre (i + 0.5, j + 0.5); UnProj uses the pixel's
    surface depth z = depth / alpha (the rasterizer's depth is the
    alpha-blended view z, not normalised), and a pixel has geometry only
    where alpha >= float32(1/255); elsewhere V = 0 and the pixel is not
    warped;
  * UnProj(x, P) = R^T (z ((u - cx)/fx, (v - cy)/fy, 1) - t) and
    Proj(X, P) = (fx X'x / X'z + cx, fy X'y / X'z + cy), X' = R X + t;
    a point behind the destination's near plane (z' < 0.2) is not warped.
The warping operator w of Eq. 13 is read as forward splatting: source pixel
x lands on the destination pixel containing (u', v') = x + V[x]; where several land on
one pixel the nearest destination depth wins, ties to the lower source
index; destination pixels nobody lands on are holes (weight 0, outputs 0).
A warped pixel carries the source colour, its destination-view depth z', its
image gradient and, when given, its normal (the normal map N of Sec. 4.2,
in source camera axes) re-expressed in the destination camera's axes,
n' = R' R^T n, evaluated as (R0i n0 + R1i n1) + R2i n2 into world axes and
((R'i0 w0 + R'i1 w1) + R'i2 w2) out of them.  Eq. 13 writes the warped gradient as
"grad V . w(G, V)", which is garbled; the reading is the chain rule through
the warp: with y = x + V(x), dI_dst/dy = (I + dV/dx)^-T dI_src/dx, the
Jacobian dV/dx by central differences over the source grid (one-sided
where a neighbour is outside the image or has no geometry, zero where
both are missing).
"""

from __future__ import annotations

import numpy as np

ALPHA_MIN = float(np.float32(1.0 / 255.0))
NEAR = 0.2


def _cam(cam):
    R = np.asarray(cam.R_wc, dtype=np.float64).reshape(3, 3)
    t = np.asarray(cam.t, dtype=np.float64)
    return R, t, float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy)


def motion(src, dst, alpha, depth):
    """V [2, H, W], destination view z [H, W], geometry mask [H, W], landing
    mask [H, W] (in front of the destination's near plane), and the
    destination coordinates u', v' [H, W].  FP64 in one
    fixed order of scalar operations (element-wise NumPy, no reductions that
    may reassociate), so the landing pixel and the depth are reproducible
    bit for bit by any FP64 implementation that follows the same order:
      z   = depth / alpha
      Xc  = (((u - cx) / fx) z, ((v - cy) / fy) z, z)
      Xw_i = (R0i (Xc0 - t0) + R1i (Xc1 - t1)) + R2i (Xc2 - t2)
      Xd_i = ((Ri0' Xw0 + Ri1' Xw1) + Ri2' Xw2) + t_i'
      u'  = fx' (Xd0 / Xd2) + cx',  v' = fy' (Xd1 / Xd2) + cy'."""
    Rs, ts, fxs, fys, cxs, cys = _cam(src)
    Rd, td, fxd, fyd, cxd, cyd = _cam(dst)
    H, W = alpha.shape
    U, Vv = np.meshgrid(np.arange(W) + 0.5, np.arange(H) + 0.5)
    a64 = np.asarray(alpha, np.float32).astype(np.float64)
    d64 = np.asarray(depth, np.float32).astype(np.float64)
    geom = np.asarray(alpha, np.float32) >= np.float32(ALPHA_MIN)
    z = np.where(geom, d64 / np.where(geom, a64, 1.0), 1.0)
    xc0 = ((U - cxs) / fxs) * z
    xc1 = ((Vv - cys) / fys) * z
    xc2 = z
    e0, e1, e2 = xc0 - ts[0], xc1 - ts[1], xc2 - ts[2]
    xw = [(Rs[0, i] * e0 + Rs[1, i] * e1) + Rs[2, i] * e2 for i in range(3)]
    xd = [((Rd[i, 0] * xw[0] + Rd[i, 1] * xw[1]) + Rd[i, 2] * xw[2]) + td[i] for i in range(3)]
    zd = xd[2]
    ok = geom & (zd >= NEAR)
    zs = np.where(ok, zd, 1.0)
    ud = fxd * (xd[0] / zs) + cxd
    vd = fyd * (xd[1] / zs) + cyd
    V = np.where(geom, np.stack([ud - U, vd - Vv]), 0.0)
    return V, np.where(ok, zd, 0.0), geom, ok, ud, vd


def jacobian(V, geom, points=None):
    """dV/dx [H, W, 2, 2] (rows: Vx, Vy; columns: d/dx, d/dy) by central
    differences over pixels with geometry; with points = (j, i) index arrays,
    only at those pixels ([n, 2, 2])."""
    H, W = geom.shape
    if points is None:
        jj, ii = np.nonzero(geom)
    else:
        jj, ii = (np.asarray(a).reshape(-1) for a in points)
    Jp = np.zeros((jj.size, 2, 2))
    for n, (j, i) in enumerate(zip(jj.tolist(), ii.tolist())):
        if not geom[j, i]:
            continue
        for axis, (di, dj) in enumerate(((1, 0), (0, 1))):
            ip, jp, im, jm = i + di, j + dj, i - di, j - dj
            hp = 0 <= ip < W and 0 <= jp < H and geom[jp, ip]
            hm = 0 <= im < W and 0 <= jm < H and geom[jm, im]
            if hp and hm:
                d = (V[:, jp, ip] - V[:, jm, im]) / 2.0
            elif hp:
                d = V[:, jp, ip] - V[:, j, i]
            elif hm:
                d = V[:, j, i] - V[:, jm, im]
            else:
                d = np.zeros(2)
            Jp[n, :, axis] = d
    if points is not None:
        return Jp
    J = np.zeros((H, W, 2, 2))
    J[jj, ii] = Jp
    return J


def warp_gradient(Jx, gx, gy):
    """The chain rule through the warp y = x + V(x): the destination gradient
    (I + dV/dx)^-T applied to the source gradient, for one pixel's Jacobian
    Jx [2, 2] and its per-channel gradients gx, gy [C].  Where I + dV/dx is
    singular the motion field folds and no gradient is defined: zeros."""
    A = np.eye(2) + Jx
    try:
        Minv_T = np.linalg.inv(A).T
    except np.linalg.LinAlgError:
        return np.zeros_like(gx), np.zeros_like(gy)
    g = Minv_T @ np.stack([gx, gy])   # [2, C]
    return g[0], g[1]


def rotate_normals(src, dst, normal):
    """Normals [3, ...] in source camera axes -> destination camera axes."""
    Rs, Rd = _cam(src)[0], _cam(dst)[0]
    n = np.asarray(normal, np.float64)
    w = [(Rs[0, i] * n[0] + Rs[1, i] * n[1]) + Rs[2, i] * n[2] for i in range(3)]
    return np.stack([((Rd[i, 0] * w[0] + Rd[i, 1] * w[1]) + Rd[i, 2] * w[2]) for i in range(3)])


def warp(src, dst, rgb, alpha, depth, dcdx, dcdy, dst_width, dst_height, normal=None):
    """Forward warp to the destination camera.  Returns dict with motion
    [2, H, W], rgb [3, H', W'], depth (destination z) [H', W'], dcdx, dcdy
    [3, H', W'], weight [H', W'] (1 where a source pixel landed), the
    winning source index [H', W'] (-1 for holes) and, when a normal map
    [3, H, W] is given, the warped normals [3, H', W']."""
    rgb, dcdx, dcdy = (np.asarray(a, np.float64) for a in (rgb, dcdx, dcdy))
    H, W = alpha.shape
    V, zd, geom, ok, ud, vd = motion(src, dst, alpha, depth)
    # the destination pixel containing (u', v'); far-off coordinates are clipped first
    ti = np.floor(np.clip(ud, -1.0, dst_width + 1.0)).astype(np.int64)
    tj = np.floor(np.clip(vd, -1.0, dst_height + 1.0)).astype(np.int64)
    land = ok & (ti >= 0) & (ti < dst_width) & (tj >= 0) & (tj < dst_height)
    src_idx = np.arange(H * W).reshape(H, W)
    # z-buffer: per destination pixel the minimum (float32 z', source index)
    best = np.full(dst_height * dst_width, -1, dtype=np.int64)
    bestz = np.full(dst_height * dst_width, np.inf)
    zf = zd.astype(np.float32).astype(np.float64)   # the comparison is on float32 depth bits
    for j in range(H):
        for i in range(W):
            if not land[j, i]:
                continue
            k = tj[j, i] * dst_width + ti[j, i]
            if zf[j, i] < bestz[k] or (zf[j, i] == bestz[k] and src_idx[j, i] < best[k]):
                bestz[k], best[k] = zf[j, i], src_idx[j, i]
    J = jacobian(V, geom)
    out_rgb = np.zeros((3, dst_height * dst_width))
    out_gx = np.zeros_like(out_rgb)
    out_gy = np.zeros_like(out_rgb)
    out_z = np.zeros(dst_height * dst_width)
    weight = np.zeros(dst_height * dst_width)
    for k in np.nonzero(best >= 0)[0]:
        s = best[k]
        j, i = divmod(s, W)
        out_rgb[:, k] = rgb[:, j, i]
        out_z[k] = zd[j, i]
        weight[k] = 1.0
        out_gx[:, k], out_gy[:, k] = warp_gradient(J[j, i], dcdx[:, j, i], dcdy[:, j, i])
    sh = (dst_height, dst_width)
    res = dict(motion=V, rgb=out_rgb.reshape(3, *sh), depth=out_z.reshape(sh), dcdx=out_gx.reshape(3, *sh),
               dcdy=out_gy.reshape(3, *sh), weight=weight.reshape(sh), source=best.reshape(sh))
    if normal is not None:
        nd = rotate_normals(src, dst, np.asarray(normal, np.float32).reshape(3, -1))
        out_n = np.zeros((3, dst_height * dst_width))
        hit = best >= 0
        out_n[:, hit] = nd[:, best[hit]]
        res["normal"] = out_n.reshape(3, *sh)
    return res
