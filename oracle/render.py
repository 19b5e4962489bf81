"""Whole forward pass of the oracle: projection, binning and sorting, then
tile compositing with image gradients (Sec. 3, Eq. 1-4)."""

from __future__ import annotations

import dataclasses

import numpy as np

from . import binning, composite
from . import conventions as cv
from .project import Projected, project


@dataclasses.dataclass
class OracleFrame:
    proj: Projected
    keys: np.ndarray         # sorted u64 keys
    values: np.ndarray       # sorted u32 Gaussian indices
    ranges: np.ndarray       # [tiles, 2]
    image: composite.Image | None
    width: int
    height: int
    bg: np.ndarray
    cam: object = None


def render_forward(scene, cam, bg=(0.0, 0.0, 0.0), near=cv.NEAR, dilation=cv.DILATION,
                   tiles=None, composite_all=True, track=True) -> OracleFrame:
    proj = project(scene, cam, near=near, dilation=dilation)
    keys, vals, ranges = binning.bin_and_sort(proj)
    W, H = int(cam.width), int(cam.height)
    bg = np.asarray(bg, dtype=np.float64)
    img = None
    if composite_all or tiles is not None:
        img = composite.composite_image(proj, vals, ranges, W, H, bg, tiles=tiles, track=track)
        iy, ix = np.mgrid[0:H, 0:W]
        img.nv = composite.normal_view(img.normal, cam, ix, iy)
    return OracleFrame(proj, keys, vals, ranges, img, W, H, bg, cam)
