"""Synthetic stand-ins for the paper's captured scenes.

The paper evaluates on Mip-NeRF 360, Tanks and Temples and Deep Blending
(Sec. 5.2) with trained 3DGS models; none of those is available, so every
workload here is drawn from ``numpy.random.default_rng(seed)`` in a fixed
field order.  Resolutions follow the paper's low-resolution inputs: its
4096x2160 and 2560x1440 outputs at 4x super sampling (Table 1) give
1024x540 and 640x360 rasters; 960x540 is the UHD/4 case.

Parameter layout (per Gaussian, float32, structure of arrays):
  means [N,3], log_scales [N,3], quats [N,4] as (w,x,y,z) and not
  necessarily unit, opacity_logits [N], sh [N,(d+1)^2,3] coefficient-major.

Camera: world->camera rotation ``R_wc`` (row major, OpenCV axes: x right,
y down, z forward) and translation ``t`` so that p_cam = R_wc p_world + t;
pinhole intrinsics fx, fy, cx, cy in pixels; integer width and height.
"""

from __future__ import annotations

import dataclasses
import math

import numpy as np

# Value of the degree-0 real spherical harmonic, 1/(2 sqrt(pi)).  Only used to
# turn a desired base colour U(0,1) into a DC coefficient when drawing inputs.
SH_C0_INPUT = 0.28209479177387814


@dataclasses.dataclass
class Scene:
    means: np.ndarray
    log_scales: np.ndarray
    quats: np.ndarray
    opacity_logits: np.ndarray
    sh: np.ndarray
    sh_degree: int

    @property
    def n(self) -> int:
        return int(self.means.shape[0])

    def subset(self, idx) -> "Scene":
        idx = np.asarray(idx)
        return Scene(self.means[idx].copy(), self.log_scales[idx].copy(),
                     self.quats[idx].copy(), self.opacity_logits[idx].copy(),
                     self.sh[idx].copy(), self.sh_degree)

    def copy(self) -> "Scene":
        return self.subset(np.arange(self.n))

    def nbytes(self) -> int:
        return sum(a.nbytes for a in (self.means, self.log_scales, self.quats,
                                      self.opacity_logits, self.sh))


@dataclasses.dataclass
class Camera:
    R_wc: np.ndarray  # [3,3] float64
    t: np.ndarray     # [3] float64
    fx: float
    fy: float
    cx: float
    cy: float
    width: int
    height: int

    def replace(self, **kw) -> "Camera":
        return dataclasses.replace(self, **kw)


def pinhole(width: int, height: int, fov_deg: float = 60.0):
    """Square pixels, horizontal field of view, principal point at the image
    centre.  Returns (fx, fy, cx, cy)."""
    f = (0.5 * width) / math.tan(math.radians(fov_deg) * 0.5)
    return f, f, 0.5 * width, 0.5 * height


def identity_camera(width: int, height: int, fov_deg: float = 60.0) -> Camera:
    fx, fy, cx, cy = pinhole(width, height, fov_deg)
    return Camera(np.eye(3), np.zeros(3), fx, fy, cx, cy, width, height)


def look_at_camera(eye, width: int, height: int, target=(0.0, 0.0, 0.0),
                   fov_deg: float = 60.0, down=(0.0, 1.0, 0.0)) -> Camera:
    """Camera at ``eye`` looking at ``target``; image y follows ``down``
    (world +y by default, +z when the view is nearly parallel to y)."""
    eye = np.asarray(eye, dtype=np.float64)
    z = np.asarray(target, dtype=np.float64) - eye
    z = z / np.linalg.norm(z)
    d = np.asarray(down, dtype=np.float64)
    x = np.cross(d, z)
    if np.linalg.norm(x) < 1e-6:
        x = np.cross(np.array([0.0, 0.0, 1.0]), z)
    x = x / np.linalg.norm(x)
    y = np.cross(z, x)
    R = np.stack([x, y, z])
    t = -R @ eye
    fx, fy, cx, cy = pinhole(width, height, fov_deg)
    return Camera(R, t, fx, fy, cx, cy, width, height)


def crop_camera(cam: Camera, x0: int, y0: int, width: int, height: int) -> Camera:
    """The same view restricted to the window [x0,x0+width) x [y0,y0+height)."""
    return cam.replace(cx=cam.cx - x0, cy=cam.cy - y0, width=width, height=height)


def _random_rotation(rng) -> np.ndarray:
    a = rng.normal(size=(3, 3))
    q, r = np.linalg.qr(a)
    q = q * np.sign(np.diag(r))[None, :]
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    return q


def _finish(rng, means, n, sh_degree, dc=None):
    log_scales = rng.normal(-4.0, 0.5, size=(n, 3))
    quats = rng.normal(size=(n, 4))
    quats /= np.linalg.norm(quats, axis=1, keepdims=True)
    op = rng.normal(0.0, 1.0, size=n)
    k = (sh_degree + 1) ** 2
    sh = np.zeros((n, k, 3), dtype=np.float32)
    sh[:, 0, :] = (rng.uniform(0.0, 1.0, size=(n, 3)) - 0.5) / SH_C0_INPUT
    if k > 1:
        sh[:, 1:, :] = rng.normal(0.0, 0.1, size=(n, k - 1, 3))
    return Scene(np.ascontiguousarray(means, dtype=np.float32),
                 log_scales.astype(np.float32), quats.astype(np.float32),
                 op.astype(np.float32), sh, sh_degree)


def gen_cfg1(seed: int = 0, n: int = 10_000, width: int = 256, height: int = 256):
    """10k Gaussians uniform in [-1,1]^2 x [2,6] in front of an identity-pose
    camera (fov 60 deg), SH degree 0 with base colour U(0,1)."""
    rng = np.random.default_rng(seed)
    u = rng.uniform(0.0, 1.0, size=(n, 3))
    means = np.empty((n, 3))
    means[:, 0] = -1.0 + 2.0 * u[:, 0]
    means[:, 1] = -1.0 + 2.0 * u[:, 1]
    means[:, 2] = 2.0 + 4.0 * u[:, 2]
    scene = _finish(rng, means, n, 0)
    return scene, identity_camera(width, height)


def gen_clustered(seed: int, n: int, sh_degree: int = 3, n_clusters: int = 64) -> Scene:
    """Gaussians in anisotropic clusters: member g belongs to cluster g mod 64;
    centres U[-1,1]^3, per-cluster random rotation and axis stretch
    U(0.25,1.75)^3 applied to N(0, 0.3^2) offsets."""
    rng = np.random.default_rng(seed)
    centres = rng.uniform(-1.0, 1.0, size=(n_clusters, 3))
    rots = np.stack([_random_rotation(rng) for _ in range(n_clusters)])
    stretch = rng.uniform(0.25, 1.75, size=(n_clusters, 3))
    off = rng.normal(0.0, 0.3, size=(n, 3))
    cl = np.arange(n) % n_clusters
    local = off * stretch[cl]
    means = centres[cl] + np.einsum("nij,nj->ni", rots[cl], local)
    del off, local
    return _finish(rng, means, n, sh_degree)


def cfg2_camera(width: int = 960, height: int = 540) -> Camera:
    return look_at_camera((0.0, 0.0, -4.0), width, height)


def gen_cfg2(seed: int = 0, n: int = 1_000_000, width: int = 960, height: int = 540):
    return gen_clustered(seed, n, 3), cfg2_camera(width, height)


def orbit_poses(n_poses: int = 60, radius: float = 4.0):
    """Eyes on a horizontal circle, eye_k = (r sin th_k, 0, -r cos th_k)."""
    th = 2.0 * math.pi * np.arange(n_poses) / n_poses
    return [(radius * math.sin(a), 0.0, -radius * math.cos(a)) for a in th]


def gen_cfg3(seed: int = 0, n: int = 6_000_000):
    return gen_clustered(seed, n, 3), orbit_poses()


def gen_cfg4(seed: int = 0, n: int = 500_000, width: int = 960, height: int = 540):
    return gen_clustered(seed, n, 3), cfg2_camera(width, height)


def gen_target(seed: int, height: int, width: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.uniform(0.0, 1.0, size=(3, height, width)).astype(np.float32)


def sphere_poses(rng, count: int, radius: float = 4.0):
    v = rng.normal(size=(count, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    return v * radius


SERVING_RESOLUTIONS = ((320, 180), (640, 360), (960, 540), (1920, 1080))


def serving_trace(seed: int = 20, rate: float = 200.0, duration: float = 32.0,
                  n_scenes: int = 4, resolutions=SERVING_RESOLUTIONS):
    """Poisson request arrivals: list of (t_arrival_s, scene_index, (w,h), eye)."""
    rng = np.random.default_rng(seed)
    out = []
    t = 0.0
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= duration:
            break
        s = int(rng.integers(n_scenes))
        r = resolutions[int(rng.integers(len(resolutions)))]
        eye = sphere_poses(rng, 1)[0]
        out.append((t, s, r, tuple(float(e) for e in eye)))
    return out


def random_scene_small(seed: int, n: int, sh_degree: int = 3, lo=(-1.0, -1.0, 2.0),
                       hi=(1.0, 1.0, 6.0), log_scale_mean: float = -3.0,
                       log_scale_std: float = 0.5, opacity_std: float = 1.0) -> Scene:
    """Small camera-space scene for unit tests (identity pose)."""
    rng = np.random.default_rng(seed)
    lo = np.asarray(lo)
    hi = np.asarray(hi)
    means = lo + (hi - lo) * rng.uniform(0.0, 1.0, size=(n, 3))
    log_scales = rng.normal(log_scale_mean, log_scale_std, size=(n, 3))
    quats = rng.normal(size=(n, 4))
    op = rng.normal(0.0, opacity_std, size=n)
    k = (sh_degree + 1) ** 2
    sh = np.zeros((n, k, 3), dtype=np.float32)
    sh[:, 0, :] = (rng.uniform(0.0, 1.0, size=(n, 3)) - 0.5) / SH_C0_INPUT
    if k > 1:
        sh[:, 1:, :] = rng.normal(0.0, 0.2, size=(n, k - 1, 3))
    return Scene(means.astype(np.float32), log_scales.astype(np.float32),
                 quats.astype(np.float32), op.astype(np.float32), sh, sh_degree)


def image_fields(seed: int, width: int, height: int, channels: int = 3):
    """Seeded planar float32 [C, H, W] image, x-gradient and y-gradient fields
    (values U(0,1), gradients N(0, 0.1)) for the image-space kernels."""
    rng = np.random.default_rng(seed)
    img = rng.random((channels, height, width)).astype(np.float32)
    gx = rng.normal(0.0, 0.1, (channels, height, width)).astype(np.float32)
    gy = rng.normal(0.0, 0.1, (channels, height, width)).astype(np.float32)
    return img, gx, gy


def frame_fields(seed: int, width: int, height: int):
    """Seeded stand-in for one rendered frame's planes, as the motion and
    warping kernels read them: alpha and depth [H, W], rgb, dcdx, dcdy
    [3, H, W], all float32.  The surface is a tilted far plane (view z 4..8)
    with a few near discs (z 1.5..3) in front of it, so depth has
    discontinuities and pixels occlude each other after a camera move; the
    top eighth of the rows is empty (alpha 0), a band there holds alpha just
    below and just above 1/255, and disc borders are semi-transparent.
    depth is alpha times the surface z, the way an alpha-blended depth of an
    opaque surface reads."""
    rng = np.random.default_rng(seed)
    ys, xs = np.mgrid[0:height, 0:width].astype(np.float64) + 0.5
    u, v = xs / width, ys / height
    z = 4.0 + 2.0 * u + 2.0 * v * v
    alpha = np.ones((height, width))
    for _ in range(4):
        cx, cy = rng.uniform(0.15, 0.85), rng.uniform(0.25, 0.85)
        r = rng.uniform(0.06, 0.18)
        zc = rng.uniform(1.5, 3.0)
        dist = np.sqrt(((u - cx) * width / height) ** 2 + (v - cy) ** 2)
        inside = dist < r
        z = np.where(inside, zc + 0.3 * (u - cx), z)
        rim = (dist >= r) & (dist < r + 2.0 / height)
        alpha = np.where(rim, rng.uniform(0.3, 0.9, size=alpha.shape), alpha)
    top = ys < height / 8.0
    alpha = np.where(top, 0.0, alpha)
    band = (ys >= height / 8.0 - 2.0) & top
    alpha = np.where(band, rng.choice([0.0039, 0.00392, 1.0 / 255.0, 0.0040, 0.5], size=alpha.shape), alpha)
    alpha = alpha.astype(np.float32)
    depth = (alpha.astype(np.float64) * z).astype(np.float32)
    rgb, gx, gy = image_fields(seed + 1, width, height)
    return alpha, depth, rgb, gx, gy
