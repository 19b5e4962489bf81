"""MI355X (gfx950) low-resolution 3DGS rasterizer with analytic image gradients.

The rasterizer behind 3DGS^3's gradient-aware super sampling and frame
interpolation (Sec. 3, Eq. 1-4): hand-written HIP kernels in libgs3.so behind
the C ABI of include/gs3.h, with a thin ctypes binding (``abi``) and a torch
wrapper (``render``) that only supplies device memory and streams.
"""

__all__ = ["abi", "render"]
