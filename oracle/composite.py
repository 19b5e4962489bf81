"""Front-to-back alpha compositing with analytic image gradients, one tile at
a time (Sec. 3, Eq. 2, Eq. 3 and Eq. 4).

Per pixel p = (i + 0.5, j + 0.5) of tile t, starting from T = 1, C = D = 0,
dC = dT = 0, walk the tile's depth-sorted list:
  alpha'  = o * exp(-q/2),  q = [dx dy] conic [dx dy]^T,  d = mean2D - p
  alpha   = min(alpha', 0.99); skip the Gaussian when alpha < 1/255;
  T'      = T (1 - alpha); stop, without blending, when T' < 1e-4;
  C      += c alpha T,  D += z alpha T                            (Eq. 2)
  dalpha  = alpha (A dx + B dy, B dx + C dy), zero at the clamp
  dC     += c (dT alpha + T dalpha)                               (Eq. 3)
  dT      = -dalpha T + (1 - alpha) dT                            (Eq. 4)
  T       = T'
Eq. 4 leaves i = 1 undefined; the reading is T_1 = 1, dT_1 = 0.  Eq. 3 sums
over the Gaussians actually blended at the pixel.  The colour derivative
term is absent from Eq. 3 because each Gaussian's colour uses one view
direction (mean minus camera centre), so dc/dx = 0 exactly.
Outputs: rgb = C + T bg, alpha = 1 - T, depth = D, dC/dx = dC_x + bg dT_x
(and y), final T and the 1-based list position of the last blended Gaussian.
The normal map N (Sec. 4.1, 4.2) is blended with the same weights,
N += n alpha T, n the Gaussian's camera-facing normal; the background adds
nothing to it.

Several results are correct near a threshold: float32 and FP64 can take the
skip, stop or clamp decision differently for the same pair.  The tile routine
therefore reports every decision whose relative distance to its threshold is
under a guard band, and ``composite_pixel`` re-evaluates one pixel with a
chosen set of such decisions inverted.
"""

from __future__ import annotations

import dataclasses

import numpy as np

from . import conventions as cv

# relative guard bands for the three threshold decisions
BAND_SKIP = 5e-5
BAND_CLAMP = 5e-5
BAND_STOP = 2e-3


@dataclasses.dataclass
class TileOut:
    tile: int
    px: np.ndarray           # [P] pixel x index (int)
    py: np.ndarray           # [P] pixel y index
    rgb: np.ndarray          # [P,3]
    alpha: np.ndarray
    depth: np.ndarray
    dcdx: np.ndarray         # [P,3]
    dcdy: np.ndarray
    normal: np.ndarray       # [P,3]
    final_T: np.ndarray
    n_contrib: np.ndarray
    evaluated: np.ndarray    # [P] pairs whose alpha was computed
    blended: np.ndarray      # [P] pairs blended
    ambiguous: dict          # pixel slot -> list of (k, kind, relative margin)
    trace: list | None       # per list position: dict of arrays (backward)


def _tile_pixels(tile, tiles_x, W, H):
    tx, ty = tile % tiles_x, tile // tiles_x
    xs = np.arange(tx * cv.TILE, min((tx + 1) * cv.TILE, W))
    ys = np.arange(ty * cv.TILE, min((ty + 1) * cv.TILE, H))
    Y, X = np.meshgrid(ys, xs, indexing="ij")
    return X.ravel(), Y.ravel()


def composite_tile(proj, svals, ranges, tile, W, H, bg, trace=False, track=True) -> TileOut:
    bg = np.asarray(bg, dtype=np.float64)
    X, Y = _tile_pixels(tile, proj.tiles_x, W, H)
    P = X.size
    pxf = X + 0.5
    pyf = Y + 0.5
    T = np.ones(P)
    C = np.zeros((P, 3))
    D = np.zeros(P)
    Nn = np.zeros((P, 3))
    dCx = np.zeros((P, 3))
    dCy = np.zeros((P, 3))
    dTx = np.zeros(P)
    dTy = np.zeros(P)
    n = np.zeros(P, dtype=np.int64)
    done = np.zeros(P, dtype=bool)
    ev = np.zeros(P, dtype=np.int64)
    bl = np.zeros(P, dtype=np.int64)
    amb: dict = {}
    steps = [] if trace else None
    s, e = int(ranges[tile, 0]), int(ranges[tile, 1])
    for k in range(e - s):
        act = np.nonzero(~done)[0]
        if act.size == 0:
            break
        g = int(svals[s + k])
        A, B, Cc = proj.conic[g]
        dx = proj.u[g] - pxf[act]
        dy = proj.v[g] - pyf[act]
        q = (A * dx * dx + 2.0 * B * dx * dy) + Cc * dy * dy
        ap = proj.opacity[g] * np.exp(-0.5 * q)
        a = np.minimum(ap, cv.ALPHA_MAX)
        ev[act] += 1
        keep = a >= cv.ALPHA_MIN
        Tn = T[act] * (1.0 - a)
        stop = keep & (Tn < cv.T_MIN)
        blend = keep & ~stop
        if track:
            m_skip = np.abs(a - cv.ALPHA_MIN) / cv.ALPHA_MIN
            m_clamp = np.abs(ap - cv.ALPHA_MAX) / cv.ALPHA_MAX
            m_stop = np.abs(Tn - cv.T_MIN) / cv.T_MIN
            for kind, m, sel in (("skip", m_skip, np.ones_like(keep)),
                                 ("clamp", m_clamp, keep),
                                 ("stop", m_stop, keep)):
                band = {"skip": BAND_SKIP, "clamp": BAND_CLAMP, "stop": BAND_STOP}[kind]
                for i in np.nonzero(sel & (m < band))[0]:
                    amb.setdefault(int(act[i]), []).append((k, kind, float(m[i])))
        done[act[stop]] = True
        b = act[blend]
        if b.size:
            ab = a[blend]
            Tb = T[b]
            w = ab * Tb
            c = proj.rgb[g]
            C[b] += w[:, None] * c[None, :]
            D[b] += w * proj.z[g]
            Nn[b] += w[:, None] * proj.normal[g][None, :]
            dxb, dyb = dx[blend], dy[blend]
            unclamped = ap[blend] < cv.ALPHA_MAX
            dax = np.where(unclamped, ab * (A * dxb + B * dyb), 0.0)
            day = np.where(unclamped, ab * (B * dxb + Cc * dyb), 0.0)
            dCx[b] += (dTx[b] * ab + Tb * dax)[:, None] * c[None, :]
            dCy[b] += (dTy[b] * ab + Tb * day)[:, None] * c[None, :]
            dTx[b] = -dax * Tb + (1.0 - ab) * dTx[b]
            dTy[b] = -day * Tb + (1.0 - ab) * dTy[b]
            T[b] = Tb * (1.0 - ab)
            n[b] = k + 1
            bl[b] += 1
            if trace:
                steps.append(dict(k=k, g=g, pix=b, alpha=ab, T=Tb, dx=dxb, dy=dyb,
                                  unclamped=unclamped))
    rgb = C + T[:, None] * bg[None, :]
    return TileOut(tile=tile, px=X, py=Y, rgb=rgb, alpha=1.0 - T, depth=D,
                   dcdx=dCx + dTx[:, None] * bg[None, :], dcdy=dCy + dTy[:, None] * bg[None, :],
                   normal=Nn, final_T=T, n_contrib=n, evaluated=ev, blended=bl, ambiguous=amb,
                   trace=steps)


def composite_pixel(proj, svals, ranges, tile, ix, iy, bg, flips=frozenset(), at=None):
    """One pixel in plain Python, with the listed (k, kind) decisions inverted.
    ``at`` replaces the pixel centre by an arbitrary image-plane point (used to
    take finite differences of the compositor with the tile list fixed)."""
    bg = np.asarray(bg, dtype=np.float64)
    px, py = (ix + 0.5, iy + 0.5) if at is None else (float(at[0]), float(at[1]))
    T, D, dTx, dTy, n = 1.0, 0.0, 0.0, 0.0, 0
    C = np.zeros(3)
    Nn = np.zeros(3)
    dCx = np.zeros(3)
    dCy = np.zeros(3)
    s, e = int(ranges[tile, 0]), int(ranges[tile, 1])
    for k in range(e - s):
        g = int(svals[s + k])
        A, B, Cc = proj.conic[g]
        dx = proj.u[g] - px
        dy = proj.v[g] - py
        q = (A * dx * dx + 2.0 * B * dx * dy) + Cc * dy * dy
        ap = proj.opacity[g] * np.exp(-0.5 * q)
        a = min(ap, cv.ALPHA_MAX)
        skip = a < cv.ALPHA_MIN
        if (k, "skip") in flips:
            skip = not skip
        if skip:
            continue
        Tn = T * (1.0 - a)
        stop = Tn < cv.T_MIN
        if (k, "stop") in flips:
            stop = not stop
        if stop:
            break
        unclamped = ap < cv.ALPHA_MAX
        if (k, "clamp") in flips:
            unclamped = not unclamped
        dax = a * (A * dx + B * dy) if unclamped else 0.0
        day = a * (B * dx + Cc * dy) if unclamped else 0.0
        c = proj.rgb[g]
        C = C + c * (a * T)
        D += (a * T) * proj.z[g]
        Nn = Nn + proj.normal[g] * (a * T)
        dCx = dCx + c * (dTx * a + T * dax)
        dCy = dCy + c * (dTy * a + T * day)
        dTx = -dax * T + (1.0 - a) * dTx
        dTy = -day * T + (1.0 - a) * dTy
        T = Tn
        n = k + 1
    return dict(rgb=C + T * bg, alpha=1.0 - T, depth=D, dcdx=dCx + dTx * bg,
                dcdy=dCy + dTy * bg, normal=Nn, final_T=T, n_contrib=n)


@dataclasses.dataclass
class Image:
    rgb: np.ndarray          # [3,H,W]
    alpha: np.ndarray        # [H,W]
    depth: np.ndarray
    dcdx: np.ndarray         # [3,H,W]
    dcdy: np.ndarray
    normal: np.ndarray       # [3,H,W]
    nv: np.ndarray           # [H,W] normal . view (filled by render_forward)
    final_T: np.ndarray
    n_contrib: np.ndarray
    evaluated: np.ndarray    # [H,W]
    blended: np.ndarray
    ambiguous: dict          # (ix, iy) -> list of (k, kind, margin)
    tiles: list              # tile ids composited (others left at background)


def composite_image(proj, svals, ranges, W, H, bg, tiles=None, track=True) -> Image:
    n_tiles = proj.tiles_x * proj.tiles_y
    tiles = list(range(n_tiles)) if tiles is None else list(tiles)
    bg = np.asarray(bg, dtype=np.float64)
    img = Image(rgb=np.broadcast_to(bg[:, None, None], (3, H, W)).copy(),
                alpha=np.zeros((H, W)), depth=np.zeros((H, W)),
                dcdx=np.zeros((3, H, W)), dcdy=np.zeros((3, H, W)),
                normal=np.zeros((3, H, W)), nv=np.zeros((H, W)), final_T=np.ones((H, W)),
                n_contrib=np.zeros((H, W), dtype=np.int64),
                evaluated=np.zeros((H, W), dtype=np.int64),
                blended=np.zeros((H, W), dtype=np.int64), ambiguous={}, tiles=tiles)
    for t in tiles:
        out = composite_tile(proj, svals, ranges, t, W, H, bg, track=track)
        put_tile(img, out)
    return img


def put_tile(img: Image, out: TileOut):
    X, Y = out.px, out.py
    img.rgb[:, Y, X] = out.rgb.T
    img.alpha[Y, X] = out.alpha
    img.depth[Y, X] = out.depth
    img.dcdx[:, Y, X] = out.dcdx.T
    img.dcdy[:, Y, X] = out.dcdy.T
    img.normal[:, Y, X] = out.normal.T
    img.final_T[Y, X] = out.final_T
    img.n_contrib[Y, X] = out.n_contrib
    img.evaluated[Y, X] = out.evaluated
    img.blended[Y, X] = out.blended
    for slot, lst in out.ambiguous.items():
        img.ambiguous[(int(X[slot]), int(Y[slot]))] = lst


def normal_view(normal, cam, ix, iy):
    """The normal-view inner product Nv (Sec. 4.1) of a rendered normal
    vector at pixel (ix, iy) (arrays broadcast): N . v with v the unit vector
    from the pixel's surface point back to the camera, i.e. minus the unit ray
    direction ((ix + 0.5 - cx)/fx, (iy + 0.5 - cy)/fy, 1)."""
    rx = (np.asarray(ix) + 0.5 - cam.cx) / cam.fx
    ry = (np.asarray(iy) + 0.5 - cam.cy) / cam.fy
    inv = 1.0 / np.sqrt(rx * rx + ry * ry + 1.0)
    return -(normal[0] * rx + normal[1] * ry + normal[2]) * inv
