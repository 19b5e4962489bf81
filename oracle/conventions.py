"""Readings of the conventions the paper does not state (Sec. 3 builds on the
original 3DGS rasterizer without restating its constants).

Each constant below is a proposed reading; the GPU path holds its own copy of
the same values.  The three compositing thresholds are the float32 numbers
nearest 1/255, 1e-4 and 0.99, because the GPU takes those decisions in float32
against float32 constants; the oracle compares its FP64 values against the
same numbers.
"""

import numpy as np

TILE = 16                    # screen tile edge in pixels
NEAR = 0.2                   # near-plane cull on view-space z
GUARD = 1.3                  # cull when |x/z| or |y/z| exceeds GUARD x half-FOV tangent
DILATION = 0.3               # low-pass term added to both diagonal entries of the 2D covariance
SIGMA_CUT = 3.0              # radius = ceil(3 sqrt(lambda_max))
ALPHA_MIN = float(np.float32(1.0 / 255.0))   # alpha below this: Gaussian skipped
ALPHA_MAX = float(np.float32(0.99))          # alpha clamp
T_MIN = float(np.float32(1e-4))              # stop before a blend that drives T below this
COLOR_OFFSET = 0.5           # added to the SH colour before clamping at 0
