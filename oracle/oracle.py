"""Python front end of the CPU oracle (``gs_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the
benchmark's CPU-baseline leg, never by the GPU library.  It does not import
the GPU package; its only input is the seeded scene/camera data (numpy arrays
and a plain camera record).

Every function follows the steps of the 3D Gaussian-splatting rasterisation
pipeline described in Section II-B and Algorithm 1 of the paper; the C file
documents the arithmetic of each step.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gs_oracle.c")
_LIB_PATH = os.path.join(_HERE, "libgs_oracle.so")
TILE = 16

# near_flags bits
NF_NEAR_PLANE, NF_DEPTH_ROUND, NF_RADIUS, NF_MEAN_ROUND, NF_DET, NF_JCLAMP, NF_RGB = (
    1, 2, 4, 8, 16, 32, 64)
NF_KEY_DECISIONS = NF_NEAR_PLANE | NF_DEPTH_ROUND | NF_RADIUS | NF_MEAN_ROUND | NF_DET
# clamp_flags bits
CF_R, CF_G, CF_B, CF_JX, CF_JY = 1, 2, 4, 8, 16


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain C, double precision, no FMA contraction)."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp"
        cmd = ["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-shared", "-fPIC",
               _SRC, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class OraCamera(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int32), ("height", ctypes.c_int32),
                ("fx", ctypes.c_double), ("fy", ctypes.c_double),
                ("cx", ctypes.c_double), ("cy", ctypes.c_double),
                ("view", ctypes.c_double * 12), ("near_plane", ctypes.c_double),
                ("bg", ctypes.c_double * 3)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        path = build()
        L = ctypes.CDLL(path)
        P = ctypes.c_void_p
        i64, i32 = ctypes.c_int64, ctypes.c_int
        L.ora_project.argtypes = [i64, i32, P, P, P, P, P, ctypes.POINTER(OraCamera), i32] + [P] * 11
        L.ora_project.restype = i32
        L.ora_count_keys.argtypes = [i64, P]
        L.ora_count_keys.restype = i64
        L.ora_build_keys.argtypes = [i64, P, P, P, i32, P, P]
        L.ora_sort_keys.argtypes = [i64, P, P]
        L.ora_ranges.argtypes = [i64, P, i32, P]
        L.ora_blend_tiles.argtypes = [i32, i32, i64, P, P, P, P, P, P, P, P, P, P, P, P, P, P, P]
        L.ora_set_threads.argtypes = [i32]
        L.ora_set_threads.restype = None
        L.ora_get_threads.argtypes = []
        L.ora_get_threads.restype = i32
        L.ora_blend_brute.argtypes = [i32, i32, i64, P, P, P, i32, P, P, P, P, P, P, P, P, P, P, P, P]
        L.ora_backward_2d.argtypes = [i32, i32, i64, P, P, P, P, P, P, P, P, P, P, P, P, P, P, P]
        L.ora_backward_params.argtypes = [i64, i32, P, P, P, P, P, ctypes.POINTER(OraCamera)] + [P] * 10
        L.ora_sh_basis.argtypes = [P, i64, i32, P]
        L.ora_sh_basis.restype = None
        for f in ("ora_build_keys", "ora_sort_keys", "ora_ranges", "ora_blend_tiles",
                  "ora_blend_brute", "ora_backward_2d", "ora_backward_params"):
            getattr(L, f).restype = i32
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _check(rc, what):
    if rc != 0:
        raise RuntimeError(f"oracle {what} failed with code {rc}")


def make_camera(cam) -> OraCamera:
    """Camera record from any object with the scenes.Camera fields (or a dict)."""
    g = (lambda k: cam[k]) if isinstance(cam, dict) else (lambda k: getattr(cam, k))
    c = OraCamera()
    c.width, c.height = int(g("width")), int(g("height"))
    # The GPU library receives these as float32; the oracle sees the same values.
    c.fx, c.fy, c.cx, c.cy = (float(np.float32(g(k))) for k in ("fx", "fy", "cx", "cy"))
    view = np.asarray(g("view"), dtype=np.float32).reshape(12)
    for i in range(12):
        c.view[i] = float(view[i])
    c.near_plane = float(np.float32(g("near_plane")))
    bg = np.asarray(g("bg"), dtype=np.float32)
    for i in range(3):
        c.bg[i] = float(bg[i])
    return c


def _scene_arrays(scene):
    n = int(scene["n"])
    deg = int(scene["sh_degree"])
    arrs = [np.ascontiguousarray(scene[k], dtype=np.float32)
            for k in ("means", "log_scales", "quats", "opacity_logits", "sh")]
    return n, deg, arrs


def project(scene, cam, round_f32=True):
    """Per-Gaussian projection and colour (Sec. II-B(1))."""
    n, deg, (means, ls, q, ol, sh) = _scene_arrays(scene)
    c = make_camera(cam)
    out = dict(
        mean2d=np.zeros((2, n)), conic=np.zeros((3, n)), opacity=np.zeros(n),
        rgb=np.zeros((3, n)), depth=np.zeros(n), depth_bits=np.zeros(n, np.uint32),
        radius=np.zeros(n, np.int32), rect=np.zeros((4, n), np.int32),
        tiles_touched=np.zeros(n, np.uint32), clamp_flags=np.zeros(n, np.uint8),
        near_flags=np.zeros(n, np.uint8))
    rc = lib().ora_project(n, deg, _p(means), _p(ls), _p(q), _p(ol), _p(sh), ctypes.byref(c),
                           int(bool(round_f32)),
                           *[_p(out[k]) for k in ("mean2d", "conic", "opacity", "rgb", "depth",
                                                  "depth_bits", "radius", "rect", "tiles_touched",
                                                  "clamp_flags", "near_flags")])
    _check(rc, "project")
    out["n"] = n
    out["round_f32"] = bool(round_f32)
    return out


def tiles_xy(width, height):
    return (width + TILE - 1) // TILE, (height + TILE - 1) // TILE


def keys_unsorted(proj, width):
    """One (tile << 32 | depth bits) key per covered tile, ascending Gaussian index."""
    n = proj["n"]
    K = int(lib().ora_count_keys(n, _p(proj["tiles_touched"])))
    keys = np.zeros(K, np.uint64)
    vals = np.zeros(K, np.uint32)
    _check(lib().ora_build_keys(n, _p(proj["rect"]), _p(proj["tiles_touched"]),
                                _p(proj["depth_bits"]), tiles_xy(width, 1)[0],
                                _p(keys), _p(vals)), "build_keys")
    return keys, vals


def sort_keys(keys, vals):
    k = np.array(keys, dtype=np.uint64, copy=True)
    v = np.array(vals, dtype=np.uint32, copy=True)
    _check(lib().ora_sort_keys(k.size, _p(k), _p(v)), "sort_keys")
    return k, v


def ranges(sorted_keys, width, height):
    tx, ty = tiles_xy(width, height)
    r = np.zeros((tx * ty, 2), np.uint32)
    _check(lib().ora_ranges(sorted_keys.size, _p(sorted_keys), tx * ty, _p(r)), "ranges")
    return r


def inverse_depth(proj):
    """1 / depth per Gaussian (0 where culled): the channel composited into
    the expected inverse depth.  With the float32-rounded projection the depth
    is rounded to float32 first, as the pipeline stores it."""
    d = proj["depth"].astype(np.float32).astype(np.float64) if proj.get("round_f32") else proj["depth"]
    vis = proj["radius"] > 0
    out = np.zeros(proj["n"])
    out[vis] = 1.0 / d[vis]
    return out


def set_threads(n):
    """Threads of the oracle's OpenMP loops from now on."""
    lib().ora_set_threads(int(n))


def get_threads():
    return int(lib().ora_get_threads())


def blend_tiles(proj, rng, point_list, cam, invdepth=None, n_eval=None):
    """Tile-list blend; with `invdepth` (an [H, W] array) also the expected
    inverse depth; with `n_eval` (an [H, W] uint32 array) the number of list
    entries each pixel examines (through the one that stops it, else all)."""
    c = make_camera(cam)
    W, H, n = c.width, c.height, proj["n"]
    bg = np.array([c.bg[0], c.bg[1], c.bg[2]])
    img = np.zeros((3, H, W))
    T = np.zeros((H, W))
    nc = np.zeros((H, W), np.uint32)
    margins = np.zeros((3, H, W))
    used = np.zeros((H, W), np.uint32)
    invd = inverse_depth(proj) if invdepth is not None else None
    _check(lib().ora_blend_tiles(W, H, n, _p(np.ascontiguousarray(rng, np.uint32)),
                                 _p(np.ascontiguousarray(point_list, np.uint32)),
                                 _p(proj["mean2d"]), _p(proj["conic"]), _p(proj["opacity"]),
                                 _p(proj["rgb"]), _p(bg), _p(img), _p(T), _p(nc), _p(margins),
                                 _p(used), _p(invd), _p(invdepth), _p(n_eval)),
           "blend_tiles")
    return img, T, nc, margins, used


def blend_brute(proj, cam, tile_filter=True, invdepth=None):
    """Every pixel against every visible Gaussian in (depth, index) order;
    with `invdepth` (an [H, W] array) also the expected inverse depth."""
    c = make_camera(cam)
    W, H, n = c.width, c.height, proj["n"]
    bg = np.array([c.bg[0], c.bg[1], c.bg[2]])
    img = np.zeros((3, H, W))
    T = np.zeros((H, W))
    nc = np.zeros((H, W), np.uint32)
    margins = np.zeros((3, H, W))
    used = np.zeros((H, W), np.uint32)
    _check(lib().ora_blend_brute(W, H, n, _p(proj["radius"]), _p(proj["rect"]),
                                 _p(proj["depth_bits"]), int(bool(tile_filter)),
                                 _p(proj["mean2d"]), _p(proj["conic"]), _p(proj["opacity"]),
                                 _p(proj["rgb"]), _p(bg), _p(img), _p(T), _p(nc), _p(margins),
                                 _p(used), _p(inverse_depth(proj) if invdepth is not None else None),
                                 _p(invdepth)),
           "blend_brute")
    return img, T, nc, margins, used


def render(scene, cam, round_f32=True):
    """Whole forward pipeline.  Returns every intermediate plus the image."""
    g = (lambda k: cam[k]) if isinstance(cam, dict) else (lambda k: getattr(cam, k))
    W, H = int(g("width")), int(g("height"))
    proj = project(scene, cam, round_f32)
    k0, v0 = keys_unsorted(proj, W)
    ks, vs = sort_keys(k0, v0)
    rg = ranges(ks, W, H)
    invdepth = np.zeros((H, W))
    n_eval = np.zeros((H, W), np.uint32)
    img, T, nc, margins, used = blend_tiles(proj, rg, vs, cam, invdepth=invdepth, n_eval=n_eval)
    return dict(proj=proj, keys_unsorted=k0, vals_unsorted=v0, keys=ks, vals=vs, ranges=rg,
                image=img, final_T=T, n_contrib=nc, margins=margins, n_used=used, K=int(ks.size),
                invdepth=invdepth, n_eval=n_eval)


def backward(scene, cam, dL_dout, fwd=None, round_f32=True, dL_dinvdepth=None):
    """Exact gradients of sum(dL_dout * image) (+ sum(dL_dinvdepth *
    invdepth)) w.r.t. every raw parameter."""
    n, deg, (means, ls, q, ol, sh) = _scene_arrays(scene)
    if fwd is None:
        fwd = render(scene, cam, round_f32)
    c = make_camera(cam)
    W, H = c.width, c.height
    bg = np.array([c.bg[0], c.bg[1], c.bg[2]])
    proj = fwd["proj"]
    g2 = dict(mean2d=np.zeros((2, n)), conic=np.zeros((3, n)), opacity=np.zeros(n),
              rgb=np.zeros((3, n)))
    dl = np.ascontiguousarray(dL_dout, dtype=np.float64).reshape(3, H, W)
    dld = invd = None
    if dL_dinvdepth is not None:
        dld = np.ascontiguousarray(dL_dinvdepth, dtype=np.float64).reshape(H, W)
        invd = inverse_depth(proj)
        g2["invdepth"] = np.zeros(n)
    _check(lib().ora_backward_2d(W, H, n, _p(fwd["ranges"]), _p(fwd["vals"]), _p(proj["mean2d"]),
                                 _p(proj["conic"]), _p(proj["opacity"]), _p(proj["rgb"]), _p(bg),
                                 _p(dl), _p(g2["mean2d"]), _p(g2["conic"]), _p(g2["opacity"]),
                                 _p(g2["rgb"]), _p(invd), _p(dld), _p(g2.get("invdepth"))), "backward_2d")
    kb = (deg + 1) ** 2
    gp = dict(means=np.zeros((3, n)), log_scales=np.zeros((3, n)), quats=np.zeros((4, n)),
              opacity_logits=np.zeros(n), sh=np.zeros((kb, 3, n)))
    _check(lib().ora_backward_params(n, deg, _p(means), _p(ls), _p(q), _p(ol), _p(sh),
                                     ctypes.byref(c), _p(g2["mean2d"]), _p(g2["conic"]),
                                     _p(g2["opacity"]), _p(g2["rgb"]), _p(gp["means"]),
                                     _p(gp["log_scales"]), _p(gp["quats"]),
                                     _p(gp["opacity_logits"]), _p(gp["sh"]), _p(g2.get("invdepth"))),
           "backward_params")
    gp["grad2d"] = g2
    return gp


def sh_basis(dirs, degree=3):
    d = np.ascontiguousarray(dirs, dtype=np.float64).reshape(-1, 3)
    out = np.zeros((d.shape[0], 16))
    lib().ora_sh_basis(_p(d), d.shape[0], degree, _p(out))
    return out


def l1_loss_grad(image, target):
    """dL/d(image) of L = mean |image - target| over the 3*H*W values."""
    return np.sign(np.asarray(image, np.float64) - target) / image.size


def flip_eligible_pixels(margins, n_used, tol_power=1e-9, tol_alpha=4e-6):
    """Pixels where a blending decision (Alg. 1: skip at power > 0, skip at
    alpha < 1/255, stop at T (1 - alpha) < 1e-4) sits so close to its
    threshold that an independent float32 evaluation may legitimately take the
    other branch.  Margins are relative distances to the threshold (the
    smallest over a pixel's examined splats).

    - power: its sign is taken in float64 from the same float32 inputs on any
      faithful implementation, so only rounding of ~1e-16 relative separates
      two evaluations; 1e-9 leaves a wide allowance.
    - alpha: a float32 evaluation of o exp(power) near 1/255 carries the
      rounding of the exponent (|log2 e * power| <= 8 there: <= 4.8e-7
      absolute, 3.3e-7 relative in exp), an exp of about 1 ulp and the
      product's half ulp, about 5e-7 relative in all; 4e-6 allows 8x that.
    - T: a float32 product over n blended splats drifts by up to ~n ulp;
      1e-6 + 3e-7 n relative.
    """
    tol_T = 1e-6 + 3e-7 * np.asarray(n_used, np.float64)
    return (margins[0] < tol_power) | (margins[1] < tol_alpha) | (margins[2] < tol_T)
