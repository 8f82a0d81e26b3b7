"""Seeded synthetic inputs: Gaussian scenes, cameras and target images.

This module only draws random numbers and builds camera poses.  It holds none
of the rendering arithmetic (no projection, no spherical-harmonics evaluation,
no blending), so both the CPU oracle and the GPU library can consume its output
without sharing any of the method's code.

Scenes stand in for the trained Mip-NeRF360 / Dr Johnson captures the paper
measures on (Section V-A, "Datasets"), which are not available here.  Every
array is float32, structure-of-arrays:

    means          [3][N]          world-space centres
    log_scales     [3][N]          per-axis log standard deviations
    quats          [4][N]          (w, x, y, z), not normalised
    opacity_logits [N]
    sh             [(deg+1)^2][3][N]   coefficient-major, then channel

Cameras are pinhole, world->camera rotation R and translation t (row-major
3x4 ``view``), camera looking down +z with image x to the right and y down,
pixel (x, y) sampled at integer coordinates, principal point at the image
centre ((W-1)/2, (H-1)/2).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

__all__ = [
    "Camera",
    "make_camera_lookat",
    "orbit_camera",
    "random_scene",
    "scene_c1",
    "scene_outdoor",
    "scene_room_like",
    "scene_fd_subcase",
    "config_scene",
    "target_image",
    "serving_scene_sizes",
    "serving_requests",
    "CONFIGS",
]


@dataclasses.dataclass
class Camera:
    width: int
    height: int
    fx: float
    fy: float
    cx: float
    cy: float
    view: np.ndarray  # float32 [3][4], world -> camera
    near_plane: float = 0.2
    bg: tuple = (0.0, 0.0, 0.0)

    def as_dict(self):
        return dataclasses.asdict(self)


def _focal_from_fovx(width: int, fovx_deg: float) -> float:
    return 0.5 * width / math.tan(math.radians(fovx_deg) * 0.5)


def make_camera_lookat(position, width, height, fovx_deg=60.0, target=(0.0, 0.0, 0.0),
                       near_plane=0.2, bg=(0.0, 0.0, 0.0)) -> Camera:
    """Pinhole camera at ``position`` looking at ``target``; world -y is image up."""
    c = np.asarray(position, dtype=np.float64)
    z = np.asarray(target, dtype=np.float64) - c
    z /= np.linalg.norm(z)
    down = np.array([0.0, -1.0, 0.0])
    x = np.cross(z, down)
    if np.linalg.norm(x) < 1e-9:  # looking straight up/down
        x = np.array([1.0, 0.0, 0.0])
    x /= np.linalg.norm(x)
    y = np.cross(z, x)
    rot = np.stack([x, y, z], axis=0)
    t = -rot @ c
    view = np.concatenate([rot, t[:, None]], axis=1).astype(np.float32)
    f = _focal_from_fovx(width, fovx_deg)
    return Camera(width=int(width), height=int(height), fx=float(np.float32(f)),
                  fy=float(np.float32(f)), cx=(width - 1) * 0.5, cy=(height - 1) * 0.5,
                  view=view, near_plane=near_plane, bg=tuple(float(b) for b in bg))


def orbit_camera(width, height, radius=4.0, azimuth_deg=0.0, elevation_deg=0.0,
                 fovx_deg=60.0, bg=(0.0, 0.0, 0.0)) -> Camera:
    """Camera on a sphere of ``radius`` around the origin, looking at the origin.

    Azimuth 0 and elevation 0 put the camera on the -z axis.
    """
    a = math.radians(azimuth_deg)
    e = math.radians(elevation_deg)
    pos = (radius * math.sin(a) * math.cos(e), -radius * math.sin(e),
           -radius * math.cos(a) * math.cos(e))
    return make_camera_lookat(pos, width, height, fovx_deg=fovx_deg, bg=bg)


def _unit_quats(rng, n):
    q = rng.standard_normal((4, n))
    q /= np.linalg.norm(q, axis=0, keepdims=True)
    return q


def _uniform_ball(rng, n, radius):
    d = rng.standard_normal((3, n))
    d /= np.linalg.norm(d, axis=0, keepdims=True)
    r = radius * rng.random(n) ** (1.0 / 3.0)
    return d * r


def _uniform_shell(rng, n, r0, r1):
    d = rng.standard_normal((3, n))
    d /= np.linalg.norm(d, axis=0, keepdims=True)
    u = rng.random(n)
    r = (r0 ** 3 + u * (r1 ** 3 - r0 ** 3)) ** (1.0 / 3.0)
    return d * r


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def random_scene(rng, n, sh_degree, means, log_scale_mu, log_scale_sigma,
                 opacity_mu, opacity_sigma, dc_low=0.0, dc_high=1.0, rest_sigma=0.3):
    k = (sh_degree + 1) ** 2
    sh = np.empty((k, 3, n))
    sh[0] = rng.uniform(dc_low, dc_high, size=(3, n))
    if k > 1:
        sh[1:] = rng.normal(0.0, rest_sigma, size=(k - 1, 3, n))
    return {
        "n": n,
        "sh_degree": sh_degree,
        "means": _f32(means),
        "log_scales": _f32(rng.normal(log_scale_mu, log_scale_sigma, size=(3, n))),
        "quats": _f32(_unit_quats(rng, n)),
        "opacity_logits": _f32(rng.normal(opacity_mu, opacity_sigma, size=n)),
        "sh": _f32(sh),
    }


def scene_c1(seed=1, n=10_000):
    """10k Gaussians in [-1,1]^3, log-scales N(-3.5,0.5), SH degree 0.

    The DC coefficient is drawn from U(-sqrt(pi), sqrt(pi)), the range that the
    degree-0 band maps onto colours U(0, 1).
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    means = rng.uniform(-1.0, 1.0, size=(3, n))
    s = math.sqrt(math.pi)
    return random_scene(rng, n, 0, means, -3.5, 0.5, 0.0, 1.0, dc_low=-s, dc_high=s)


def scene_outdoor(seed, n, ball_radius=3.0, sh_degree=3, log_scale_mu=-4.0,
                  log_scale_sigma=1.0, opacity_mu=0.5, opacity_sigma=1.5):
    """Unbounded-outdoor-like scene: 75% in a ball, 25% in a shell of radius 20-60."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n_ball = (3 * n) // 4
    means = np.concatenate([_uniform_ball(rng, n_ball, ball_radius),
                            _uniform_shell(rng, n - n_ball, 20.0, 60.0)], axis=1)
    return random_scene(rng, n, sh_degree, means, log_scale_mu, log_scale_sigma,
                        opacity_mu, opacity_sigma)


def scene_room_like(seed=7, n=1_000_000):
    """Blend-bound scene shaped like the paper's profiled room capture (Table 3)."""
    return scene_outdoor(seed, n, log_scale_mu=-5.0, log_scale_sigma=0.8,
                         opacity_mu=-1.0, opacity_sigma=1.5)


def scene_fd_subcase(seed=41, n=500, sh_degree=3):
    """Small ball-distributed scene for finite-difference gradient checks."""
    rng = np.random.Generator(np.random.PCG64(seed))
    means = _uniform_ball(rng, n, 3.0)
    return random_scene(rng, n, sh_degree, means, -2.5, 0.5, 0.5, 1.5)


# name -> (scene factory, (width, height), camera factory)
CONFIGS = {
    "c1": dict(scene=lambda: scene_c1(1), size=(256, 256),
               camera=lambda: make_camera_lookat((0.0, 0.0, -4.0), 256, 256)),
    "c2": dict(scene=lambda: scene_outdoor(2, 3_000_000), size=(1237, 822),
               camera=lambda: orbit_camera(1237, 822, 4.0, 0.0, 0.0)),
    "c3": dict(scene=lambda: scene_outdoor(3, 6_000_000, ball_radius=5.0), size=(1920, 1080),
               camera=lambda: orbit_camera(1920, 1080, 4.0, 0.0, 0.0)),
    "c4": dict(scene=lambda: scene_outdoor(4, 1_000_000), size=(1280, 720),
               camera=lambda: orbit_camera(1280, 720, 4.0, 0.0, 0.0)),
    "room": dict(scene=lambda: scene_room_like(7), size=(778, 519),
                 camera=lambda: orbit_camera(778, 519, 4.0, 0.0, 0.0)),
}


def config_scene(name, n=None, seed=None):
    """Scene and camera of a named configuration.  ``n`` shrinks the scene
    (same distribution, same seed) for quick runs."""
    cfg = CONFIGS[name]
    if n is None and seed is None:
        scene = cfg["scene"]()
    elif name == "c1":
        scene = scene_c1(seed if seed is not None else 1, n or 10_000)
    elif name == "room":
        scene = scene_room_like(seed if seed is not None else 7, n or 1_000_000)
    else:
        default = {"c2": (2, 3_000_000, 3.0), "c3": (3, 6_000_000, 5.0),
                   "c4": (4, 1_000_000, 3.0)}[name]
        scene = scene_outdoor(seed if seed is not None else default[0], n or default[1],
                              ball_radius=default[2])
    return scene, cfg["camera"]()


def target_image(seed, width, height):
    """Seeded U(0,1) target image, planar [3][H][W] float32."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return _f32(rng.random((3, height, width)))


SERVING_RESOLUTIONS = ((640, 360), (1280, 720), (1237, 822), (1920, 1080))


def serving_scene_sizes(seed=5, count=16, lo=200_000, hi=3_000_000):
    rng = np.random.Generator(np.random.PCG64(seed))
    return [int(round(math.exp(v))) for v in rng.uniform(math.log(lo), math.log(hi), size=count)]


def serving_requests(seed, count, n_scenes, rate_per_s):
    """Poisson arrivals: (arrival_s, scene_id, width, height, azimuth, elevation)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    gaps = rng.exponential(1.0 / rate_per_s, size=count)
    t = np.cumsum(gaps) - gaps[0]
    out = []
    for i in range(count):
        w, h = SERVING_RESOLUTIONS[int(rng.integers(0, len(SERVING_RESOLUTIONS)))]
        out.append((float(t[i]), int(rng.integers(0, n_scenes)), w, h,
                    float(rng.uniform(0.0, 360.0)), float(rng.uniform(-15.0, 15.0))))
    return out
