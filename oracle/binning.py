"""Tile binning and depth sorting (Sec. 3: the 2D Gaussians are depth-sorted
before blending; the tile grid is the 3DGS rasterizer's 16x16 screen tiles).

Reading of "depth-sorted": each (Gaussian, covered tile) pair gets the 64-bit
key (tile_id << 32) | float32_bits(view z), tile_id = ty * tiles_x + tx,
emitted for Gaussians in index order, rows ty then columns tx.  Pairs are
ordered by (key, Gaussian index): equal float32 depths keep index order.
Per-tile lists are the half-open ranges of the sorted array; an empty tile
has the range [0, 0).
"""

from __future__ import annotations

import numpy as np


def emit_keys(proj):
    """Keys and values in emission order (library routines: repeat, cumsum)."""
    g = np.nonzero(proj.touched > 0)[0]
    cnt = proj.touched[g]
    total = int(cnt.sum())
    gi = np.repeat(g, cnt)
    start = np.repeat(np.cumsum(cnt) - cnt, cnt)
    local = np.arange(total, dtype=np.int64) - start
    rect = proj.rect[gi]
    w = rect[:, 2] - rect[:, 0] + 1
    ty = rect[:, 1] + local // w
    tx = rect[:, 0] + local % w
    tile = ty * proj.tiles_x + tx
    zk = proj.zkey[gi].astype(np.uint64)
    keys = (tile.astype(np.uint64) << np.uint64(32)) | zk
    return keys, gi.astype(np.uint32)


def sort_pairs(keys, values):
    """Lexicographic (key, value) order; a library sort is the step here."""
    order = np.lexsort((values, keys))
    return keys[order], values[order]


def tile_ranges(sorted_keys, n_tiles: int):
    tiles = (sorted_keys >> np.uint64(32)).astype(np.int64)
    ids = np.arange(n_tiles)
    first = np.searchsorted(tiles, ids, side="left")
    last = np.searchsorted(tiles, ids, side="right")
    ranges = np.stack([first, last], axis=1).astype(np.int64)
    ranges[first == last] = 0
    return ranges


def bin_and_sort(proj):
    keys, vals = emit_keys(proj)
    skeys, svals = sort_pairs(keys, vals)
    ranges = tile_ranges(skeys, proj.tiles_x * proj.tiles_y)
    return skeys, svals, ranges
