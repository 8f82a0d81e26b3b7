"""Pins of the oracle's expected inverse depth (the optional output of the
Appendix B blend kernels: sum over blended splats of alpha T / depth) and of
its gradient."""
import numpy as np

from oracle import oracle as O
from paper_2509_25626_amd import scenes as S
from tests.helpers import axis_camera, mk_scene

SH_C0 = 0.28209479177387814


def _random_scene(n, seed, z=None):
    rng = np.random.Generator(np.random.PCG64(seed))
    means = rng.uniform(-0.8, 0.8, (3, n))
    if z is not None:
        means[2] = z  # every Gaussian at the same camera depth (axis camera: depth = z + 4)
    sc = S.random_scene(rng, n, 0, means, -2.0, 0.4, 0.5, 1.2)
    return sc


def test_equal_depths_give_coverage_over_depth():
    # all splats at one depth z: sum a_i T_i = 1 - T_final, so D = (1 - T_final) / z
    sc = _random_scene(60, 3, z=0.25)
    cam = axis_camera(48, 40, f=40.0)
    r = O.render(sc, cam, round_f32=False)
    z = r["proj"]["depth"][r["proj"]["radius"] > 0]
    assert np.allclose(z, z[0], rtol=0, atol=1e-12)
    assert (r["n_used"] > 0).sum() > 100
    assert np.allclose(r["invdepth"], (1.0 - r["final_T"]) / z[0], rtol=0, atol=1e-12)


def test_inverse_depth_is_a_colour_channel_with_black_background():
    # with rgb_i = 1 / depth_i (degree-0 SH) and a black background the red
    # channel composites exactly what the inverse depth does
    sc = _random_scene(80, 4)
    cam = axis_camera(40, 36, f=35.0)
    p = O.project(sc, cam, round_f32=False)
    vis = p["radius"] > 0
    dc = np.zeros(sc["n"])
    dc[vis] = (1.0 / p["depth"][vis] - 0.5) / SH_C0
    sh = sc["sh"].copy()
    sh[0, 0] = dc.astype(np.float32)
    sc2 = dict(sc, sh=sh)
    r = O.render(sc2, cam, round_f32=False)
    assert (r["n_used"] > 0).sum() > 100
    # DC is stored as float32: the colours are 1/depth to ~6e-8 relative
    assert np.allclose(r["image"][0], r["invdepth"], rtol=1e-6, atol=1e-9)


def test_tile_path_equals_brute_force():
    sc = _random_scene(200, 5)
    cam = axis_camera(64, 48, f=50.0)
    r = O.render(sc, cam, round_f32=True)
    d = np.zeros((48, 64))
    O.blend_brute(r["proj"], cam, tile_filter=True, invdepth=d)
    assert np.array_equal(d, r["invdepth"])
    assert np.abs(r["invdepth"]).max() > 0


def _step(x0):
    import math
    e = math.floor(math.log2(max(abs(x0), 0.25))) - 17
    h = 2.0 ** e
    up, dn = np.float32(x0 + h), np.float32(x0 - h)
    if float(up) - x0 != h or x0 - float(dn) != h:
        return None, None, None
    return h, up, dn


def _sig(r):
    p = r["proj"]
    return (p["radius"].tobytes(), p["rect"].tobytes(), r["n_contrib"].tobytes(), r["n_used"].tobytes(),
            p["clamp_flags"].tobytes())


def test_fd_gradient_through_inverse_depth():
    # L = sum(w * image) + sum(wd * invdepth): central differences of the
    # double-precision forward against the analytic backward, every parameter
    rng = np.random.Generator(np.random.PCG64(6))
    n = 10
    means = rng.uniform(-0.8, 0.8, (3, n))
    sc = S.random_scene(rng, n, 1, means, -1.7, 0.35, 0.3, 1.0)
    cam = axis_camera(30, 26, f=28.0, bg=(0.2, 0.4, 0.1))
    w = rng.normal(size=(3, 26, 30))
    wd = rng.normal(size=(26, 30)) * 3.0

    def loss(s):
        r = O.render(s, cam, round_f32=False)
        return float((r["image"] * w).sum() + (r["invdepth"] * wd).sum()), r

    L0, base = loss(sc)
    g = O.backward(sc, cam, w, fwd=base, round_f32=False, dL_dinvdepth=wd)
    g_nod = O.backward(sc, cam, w, fwd=base, round_f32=False)
    assert np.abs(g["means"] - g_nod["means"]).max() > 1e-6  # the depth term reaches the means
    checked = 0
    for name in ("means", "log_scales", "quats", "opacity_logits", "sh"):
        gmax = max(np.abs(g[name]).max(), 1e-12)
        for idx in range(sc[name].size):
            x0 = float(sc[name].reshape(-1)[idx])
            h, up, dn = _step(x0)
            if h is None:
                continue
            vals = []
            for v in (up, dn):
                s2 = dict(sc)
                s2[name] = sc[name].copy()
                s2[name].reshape(-1)[idx] = v
                L, r = loss(s2)
                if _sig(r) != _sig(base):
                    break
                vals.append(L)
            if len(vals) != 2:
                continue
            fd = (vals[0] - vals[1]) / (2 * h)
            an = float(g[name].reshape(-1)[idx])
            scale = max(abs(an), 1e-3 * gmax)
            assert abs(fd - an) <= 1e-5 * scale + 1e-14 * abs(L0) / h, (name, idx, fd, an)
            checked += 1
    assert checked > 150
