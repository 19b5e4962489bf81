"""Seeded synthetic inputs (scenes, cameras, loss targets, request traces).

This package is shared by the FP64 oracle, the GPU path's tests and the
benchmark.  It holds input recipes only: random draws and the camera pose
construction that places a pinhole camera in the world.  None of the
rasterizer's arithmetic (projection, colour, sorting, compositing) lives here.
"""

from .scenes import (  # noqa: F401
    Camera,
    Scene,
    SERVING_RESOLUTIONS,
    SH_C0_INPUT,
    cfg2_camera,
    crop_camera,
    gen_cfg1,
    gen_clustered,
    gen_cfg2,
    gen_cfg3,
    gen_cfg4,
    frame_fields,
    image_fields,
    gen_target,
    identity_camera,
    look_at_camera,
    orbit_poses,
    pinhole,
    random_scene_small,
    serving_trace,
    sphere_poses,
)
