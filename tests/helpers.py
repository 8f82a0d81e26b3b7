"""Small shared helpers for the test suite (scene construction only)."""
import math

import numpy as np

from paper_2509_25626_amd.scenes import Camera, make_camera_lookat


def mk_scene(means, log_scales, quats=None, opacity_logits=None, sh=None, sh_degree=0):
    means = np.asarray(means, np.float64).reshape(3, -1)
    n = means.shape[1]
    ls = np.asarray(log_scales, np.float64)
    if ls.ndim == 1 and ls.size == n:
        ls = np.tile(ls, (3, 1))
    ls = ls.reshape(3, n)
    if quats is None:
        quats = np.tile(np.array([[1.0], [0.0], [0.0], [0.0]]), (1, n))
    if opacity_logits is None:
        opacity_logits = np.zeros(n)
    k = (sh_degree + 1) ** 2
    if sh is None:
        sh = np.zeros((k, 3, n))
    return {
        "n": n, "sh_degree": sh_degree,
        "means": np.ascontiguousarray(means, np.float32),
        "log_scales": np.ascontiguousarray(ls, np.float32),
        "quats": np.ascontiguousarray(np.asarray(quats, np.float64).reshape(4, n), np.float32),
        "opacity_logits": np.ascontiguousarray(np.asarray(opacity_logits).reshape(n), np.float32),
        "sh": np.ascontiguousarray(np.asarray(sh).reshape(k, 3, n), np.float32),
    }


def axis_camera(W, H, f=None, dist=4.0, bg=(0.0, 0.0, 0.0)):
    """Camera on the -z axis at ``dist`` looking at the origin: R = I, t = (0, 0, dist)."""
    cam = make_camera_lookat((0.0, 0.0, -dist), W, H, bg=bg)
    if f is not None:
        cam.fx = cam.fy = float(np.float32(f))
    return cam


def logit(p):
    return math.log(p / (1.0 - p))


def f32(x):
    return float(np.float32(x))
