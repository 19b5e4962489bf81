"""Comparison helpers for the GPU-vs-oracle parity tests.

Images and gradient buffers must agree within TOL max-abs (float32 GPU vs
FP64 oracle).  Where float32 and FP64 may take a threshold decision (skip,
stop, clamp) differently, both results are correct: a pixel that differs is
accepted when the oracle flagged a decision on it within its guard band and
re-running the oracle with that decision (or a pair of them) inverted matches
the GPU.  Such pixels are counted and reported.
"""

from __future__ import annotations

import itertools

import numpy as np

from oracle import composite

TOL = 1e-4
FIELDS = ("rgb", "alpha", "depth", "dcdx", "dcdy", "final_T")
NORMAL_FIELDS = ("normal", "nv")


def gpu_outputs_numpy(out: dict) -> dict:
    res = {k: v.detach().cpu().numpy() for k, v in out.items() if v is not None}
    if "n_contrib" in res:
        res["n_contrib"] = res["n_contrib"].view(np.uint32).astype(np.int64)
    return res


def _dict_err(g, d, ix, iy, fields=FIELDS):
    e = 0.0
    for f in fields:
        a = g[f]
        v = np.asarray(d[f])
        if a.ndim == 3:
            e = max(e, float(np.abs(a[:, iy, ix] - v).max()))
        else:
            e = max(e, abs(float(a[iy, ix]) - float(v)))
    return e


def compare_frame(gpu: dict, frame, tiles=None, tol=TOL, max_flips=2):
    """Compare GPU outputs with the oracle's image on the composited tiles
    (and the normal maps when the GPU returned them).  Returns a stats dict;
    stats['unresolved'] lists pixels that match no correct result."""
    img = frame.image
    ref = dict(rgb=img.rgb, alpha=img.alpha, depth=img.depth, dcdx=img.dcdx, dcdy=img.dcdy,
               final_T=img.final_T, normal=img.normal, nv=img.nv)
    fields = FIELDS + (NORMAL_FIELDS if all(f in gpu for f in NORMAL_FIELDS) else ())
    P = frame.proj
    tiles = img.tiles if tiles is None else tiles
    stats = dict(pixels=0, clean_max_err=0.0, flipped=0, unresolved=[], n_contrib_mismatch=0)
    # every pixel's largest error over the fields and its n_contrib check at
    # once; only the pixels that fail either are examined one by one
    H, W = frame.height, frame.width
    err_img = np.zeros((H, W))
    for f in fields:
        d = np.abs(np.asarray(gpu[f], dtype=np.float64) - np.asarray(ref[f], dtype=np.float64))
        err_img = np.maximum(err_img, d.max(axis=0) if d.ndim == 3 else d)
    nok_img = np.asarray(gpu["n_contrib"]).astype(np.int64) == np.asarray(img.n_contrib).astype(np.int64)
    for t in tiles:
        tx, ty = t % P.tiles_x, t // P.tiles_x
        x0, x1 = tx * 16, min(tx * 16 + 16, W)
        y0, y1 = ty * 16, min(ty * 16 + 16, H)
        e_t = err_img[y0:y1, x0:x1]
        ok_t = (e_t <= tol) & nok_img[y0:y1, x0:x1]
        stats["pixels"] += int(e_t.size)
        if ok_t.any():
            stats["clean_max_err"] = max(stats["clean_max_err"], float(e_t[ok_t].max()))
        for jy, jx in zip(*np.nonzero(~ok_t)):
            iy, ix = int(y0 + jy), int(x0 + jx)
            err = float(err_img[iy, ix])
            n_ok = bool(nok_img[iy, ix])
            amb = img.ambiguous.get((ix, iy), [])
            decs = [(k, kind) for (k, kind, _) in amb]
            ok = False
            for r in range(1, max_flips + 1):
                for fl in itertools.combinations(decs, r):
                    d = composite.composite_pixel(P, frame.values, frame.ranges, t, ix, iy, frame.bg,
                                                  flips=frozenset(fl))
                    d["nv"] = composite.normal_view(d["normal"], frame.cam, ix, iy)
                    if (_dict_err(gpu, d, ix, iy, fields) <= tol
                            and int(gpu["n_contrib"][iy, ix]) == d["n_contrib"]):
                        ok = True
                        break
                if ok:
                    break
            if ok:
                stats["flipped"] += 1
            else:
                if not n_ok:
                    stats["n_contrib_mismatch"] += 1
                stats["unresolved"].append((ix, iy, err, int(gpu["n_contrib"][iy, ix]),
                                            int(img.n_contrib[iy, ix]), amb))
    return stats
