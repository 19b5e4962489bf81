"""FP64 CPU oracle for the low-resolution 3DGS rasterizer with analytic image
gradients.

TEST INFRASTRUCTURE ONLY.  Nothing in the product package imports, calls or
links this package; only the tests, the smoke check and the benchmark's CPU
baseline leg do.  It shares no code with the HIP path (no kernels, headers,
helpers, tables or constant generators); the only common module is
``synth`` (seeded input draws, no rasterizer arithmetic).

What it computes (3DGS³, Sec. 3 "Preliminaries"):
  * Eq. 1 and the R S S^T R^T factorisation: 3D Gaussian primitives;
  * EWA splatting of each primitive to a 2D image-space Gaussian;
  * depth sorting of the 2D Gaussians per 16x16 screen tile;
  * Eq. 2: front-to-back alpha blending with view-dependent SH colour;
  * Eq. 3 and Eq. 4: the analytic screen-space image gradients dI/dx, dI/dy,
    accumulated in the same front-to-back pass;
  * the per-pixel alpha-blended depth that the GASS and LTFI modules consume
    (Sec. 4.1, 4.2), and the normal map N and normal-view map Nv they also
    take (shortest-axis normals blended like colour, the RaDe-GS rendering
    of Sec. 5.1);
  * the reverse-mode adjoint of all of the above with respect to the
    Gaussian parameters (plain FP64 adjoint code, not autograd);
  * Sec. 4.1, Eq. 5-7: gradient-aware interpolation of the low-resolution
    image to S x S times its pixels with a fixed least-squares matrix
    (``oracle.upsample``);
  * Sec. 4.2, Eq. 12-13: pose-derived motion vectors and forward warping of
    the image, depth and gradient buffers to another camera
    (``oracle.warp``).

Conventions the paper leaves open are fixed in ``oracle.conventions``; each
one is a stated reading, duplicated by value (never by import) on the GPU
side.
"""

from . import conventions, sh, project, binning, composite, brute, backward, render, upsample, warp  # noqa: F401
from .render import render_forward, OracleFrame  # noqa: F401
