"""The oracle's tile compositing (Sec. 3, Eq. 2-4) spread over worker
processes, for full frames at the benchmark's sizes.

TEST INFRASTRUCTURE ONLY, like the rest of ``oracle``: the tests and the
benchmark's CPU-baseline leg use it; the product path never does.

Projection and binning stay in the calling process.  The arrays compositing
reads (2D means, conics, opacities, colours, view depths, normals, the
sorted Gaussian indices and the tile ranges) are handed to every worker once
when the pool starts; each worker then runs ``composite.composite_tile``
unchanged on the tiles it is given, so the image is the one
``composite.composite_image`` would produce, tile for tile.  Workers are
started with the "spawn" method: they begin as fresh interpreters and touch
no device state of the caller.
"""

from __future__ import annotations

import multiprocessing as mp
import os
import time
import types

import numpy as np

from . import composite

_STATE = None


def _init(state):
    global _STATE
    _STATE = state


def _run(args):
    tiles, W, H, bg, track = args
    s = _STATE
    proj = types.SimpleNamespace(conic=s["conic"], u=s["u"], v=s["v"], opacity=s["opacity"], rgb=s["rgb"],
                                 z=s["z"], normal=s["normal"], tiles_x=s["tiles_x"], tiles_y=s["tiles_y"])
    return [composite.composite_tile(proj, s["values"], s["ranges"], t, W, H, bg, track=track) for t in tiles]


def default_workers() -> int:
    return max(1, min(16, os.cpu_count() or 1))


def composite_image_parallel(proj, values, ranges, W, H, bg, tiles=None, track=True, workers=None,
                             timing=None) -> composite.Image:
    """``composite.composite_image`` over a pool of `workers` processes.
    When `timing` is a dict, it receives 'pool_start_s' (starting the
    workers and handing them the arrays) and 'composite_s' (wall time of the
    compositing itself)."""
    n_tiles = proj.tiles_x * proj.tiles_y
    tiles = list(range(n_tiles)) if tiles is None else [int(t) for t in tiles]
    bg = np.asarray(bg, dtype=np.float64)
    img = composite.Image(rgb=np.broadcast_to(bg[:, None, None], (3, H, W)).copy(),
                          alpha=np.zeros((H, W)), depth=np.zeros((H, W)),
                          dcdx=np.zeros((3, H, W)), dcdy=np.zeros((3, H, W)),
                          normal=np.zeros((3, H, W)), nv=np.zeros((H, W)), final_T=np.ones((H, W)),
                          n_contrib=np.zeros((H, W), dtype=np.int64),
                          evaluated=np.zeros((H, W), dtype=np.int64),
                          blended=np.zeros((H, W), dtype=np.int64), ambiguous={}, tiles=tiles)
    workers = default_workers() if workers is None else max(1, int(workers))
    state = dict(conic=proj.conic, u=proj.u, v=proj.v, opacity=proj.opacity, rgb=proj.rgb, z=proj.z,
                 normal=proj.normal, tiles_x=proj.tiles_x, tiles_y=proj.tiles_y,
                 values=np.ascontiguousarray(values), ranges=np.ascontiguousarray(ranges))
    # longest lists first, dealt into small chunks so the pool balances itself
    lens = np.asarray([int(ranges[t, 1]) - int(ranges[t, 0]) for t in tiles])
    order = [tiles[i] for i in np.argsort(-lens, kind="stable")]
    chunk = max(1, min(8, len(order) // (4 * workers) or 1))
    jobs = [(order[i:i + chunk], W, H, bg, track) for i in range(0, len(order), chunk)]
    t0 = time.perf_counter()
    ctx = mp.get_context("spawn")
    with ctx.Pool(workers, initializer=_init, initargs=(state,)) as pool:
        # every worker has received the arrays once this trivial round returns
        pool.map(_noop, range(workers), chunksize=1)
        t1 = time.perf_counter()
        for outs in pool.imap_unordered(_run, jobs):
            for out in outs:
                composite.put_tile(img, out)
        t2 = time.perf_counter()
    if timing is not None:
        timing["pool_start_s"] = t1 - t0
        timing["composite_s"] = t2 - t1
        timing["workers"] = workers
    return img


def _noop(_):
    return _STATE is not None
