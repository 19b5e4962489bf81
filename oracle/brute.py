"""Brute-force per-pixel renderer: an independent route to the per-tile lists.

For the tile containing a pixel, collect every Gaussian whose tile rectangle
covers that tile by scanning all Gaussians, order them by (float32 view z,
index) with Python's own sort, and composite.  No keys, no key sort and no
ranges are involved, so a mistake in key layout, emission order, sort
stability or range extraction shows up as a difference from the tile path.

``untruncated`` drops the rectangle test altogether (every visible Gaussian
in depth order).  It is not the method: the 3-sigma square cuts alpha off up
to about o * exp(-4.5) outside it, so its difference is information only.
"""

from __future__ import annotations

import numpy as np

from .composite import composite_pixel


def tile_list(proj, tile, untruncated=False):
    tx, ty = tile % proj.tiles_x, tile // proj.tiles_x
    zk = proj.zkey
    members = []
    for g in range(proj.n):
        if proj.touched[g] <= 0:
            if not (untruncated and proj.valid[g]):
                continue
        elif not untruncated:
            x0, y0, x1, y1 = proj.rect[g]
            if not (x0 <= tx <= x1 and y0 <= ty <= y1):
                continue
        members.append((int(zk[g]), g))
    members.sort()
    return np.array([g for _, g in members], dtype=np.uint32)


def render_pixel(proj, ix, iy, bg, untruncated=False, lists=None):
    tile = (iy // 16) * proj.tiles_x + (ix // 16)
    if lists is not None and tile in lists:
        lst = lists[tile]
    else:
        lst = tile_list(proj, tile, untruncated)
        if lists is not None:
            lists[tile] = lst
    ranges = np.zeros((tile + 1, 2), dtype=np.int64)
    ranges[tile] = (0, lst.size)
    return composite_pixel(proj, lst, ranges, tile, ix, iy, bg)
