"""Pins of the oracle's analytic backward pass: central finite differences of
its own double-precision forward (with every discrete decision checked to be
unchanged by the perturbation) and a single-Gaussian closed form."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2509_25626_amd import scenes as S
from tests.helpers import axis_camera, f32, logit, mk_scene

PARAMS = ("means", "log_scales", "quats", "opacity_logits", "sh")


def _signature(r):
    p = r["proj"]
    return (p["radius"].tobytes(), p["rect"].tobytes(), r["n_contrib"].tobytes(),
            r["n_used"].tobytes(), p["clamp_flags"].tobytes())


def _loss(scene, cam, w):
    r = O.render(scene, cam, round_f32=False)
    return float((r["image"] * w).sum()), r


def _step(x0):
    """A power-of-two step h ~ 8e-6 |x| with x0 +- h exactly representable in float32."""
    e = math.floor(math.log2(max(abs(x0), 0.25))) - 17
    h = 2.0 ** e
    up, dn = np.float32(x0 + h), np.float32(x0 - h)
    if float(up) - x0 != h or x0 - float(dn) != h:
        return None, None, None
    return h, up, dn


def fd_check(scene, cam, w, picks, rel=1e-5):
    base_L, base = _loss(scene, cam, w)
    absL = float(np.abs(base["image"] * w).sum())
    sig = _signature(base)
    g = O.backward(scene, cam, w, fwd=base, round_f32=False)
    gmax = {k: max(np.abs(g[k]).max(), 1e-12) for k in PARAMS}
    checked = skipped = 0
    worst = 0.0
    for name, idx in picks:
        flat = scene[name].reshape(-1)
        x0 = float(flat[idx])
        h, up, dn = _step(x0)
        if h is None:
            skipped += 1
            continue
        vals = []
        for v in (up, dn):
            sc = dict(scene)
            sc[name] = scene[name].copy()
            sc[name].reshape(-1)[idx] = v
            L, r = _loss(sc, cam, w)
            if _signature(r) != sig:
                break
            vals.append(L)
        if len(vals) != 2:
            skipped += 1  # a discrete decision moved: the loss is not differentiable here
            continue
        fd = (vals[0] - vals[1]) / (2 * h)
        an = float(g[name].reshape(-1)[idx])
        scale = max(abs(an), 1e-3 * gmax[name])
        roundoff = 1e-14 * absL / h  # double-precision noise of the two loss values
        worst = max(worst, abs(fd - an) / scale)
        assert abs(fd - an) <= rel * scale + roundoff, (name, idx, fd, an)
        checked += 1
    return checked, skipped, worst


def _tiny_scene(n=12, deg=3, seed=21):
    rng = np.random.Generator(np.random.PCG64(seed))
    means = rng.uniform(-0.9, 0.9, (3, n))
    sc = S.random_scene(rng, n, deg, means, -1.7, 0.35, 0.3, 1.0)
    return sc


def test_fd_all_parameters_tiny_scene():
    sc = _tiny_scene()
    cam = axis_camera(32, 28, f=30.0, bg=(0.3, 0.1, 0.6))
    w = np.random.default_rng(1).normal(size=(3, 28, 32))
    picks = [(name, i) for name in PARAMS for i in range(sc[name].size)]
    checked, skipped, worst = fd_check(sc, cam, w, picks)
    assert checked >= 0.9 * len(picks), (checked, skipped)


def test_fd_guard_band_and_colour_clamp_paths():
    # Gaussians beyond the 1.3x field-of-view band (clamped Jacobian) and a colour
    # channel clamped at zero: their gradients follow the decisions held fixed.
    n = 4
    # camera limit 1.3 * W / (2 f) = 1.04; x/z of Gaussians 0, 1 and y/z of Gaussian 2 ~ 1.1
    means = np.array([[4.95, -5.0, 0.2, 0.0], [0.1, 0.3, 4.95, 0.0], [0.5, 0.55, 0.5, -1.0]])
    sh = np.zeros((4, 3, n))
    sh[0] = [[0.9, 0.2, 0.5, -3.0], [0.1, 0.8, 0.4, 0.7], [0.5, 0.3, -2.0, 0.2]]
    sh[1:] = np.random.default_rng(2).normal(0, 0.3, (3, 3, n))
    q = np.random.default_rng(3).normal(size=(4, n))
    ls = np.array([[-0.2, -0.3, -0.25, -1.2], [-0.5, -0.1, -0.45, -1.5], [-0.3, -0.6, -0.2, -1.0]])
    sc = mk_scene(means, ls, quats=q, opacity_logits=[0.5, 1.0, -0.3, 0.8], sh=sh, sh_degree=1)
    cam = axis_camera(40, 40, f=25.0, bg=(0.2, 0.2, 0.2))
    p = O.project(sc, cam)
    assert p["clamp_flags"][0] & O.CF_JX and p["clamp_flags"][1] & O.CF_JX
    assert p["clamp_flags"][2] & O.CF_JY
    assert p["clamp_flags"][3] & O.CF_R
    assert (p["radius"] > 0).all()
    w = np.random.default_rng(4).normal(size=(3, 40, 40))
    picks = [(name, i) for name in PARAMS for i in range(sc[name].size)]
    checked, skipped, _ = fd_check(sc, cam, w, picks)
    assert checked >= 0.85 * len(picks), (checked, skipped)


@pytest.mark.slow
def test_fd_sampled_parameters_500_gaussian_subcase():
    # The differentiable configuration's finite-difference sub-case: 500 Gaussians, 64x64.
    sc = S.scene_fd_subcase(41, 500)
    cam = S.orbit_camera(64, 64, 4.0, 20.0, 5.0)
    w = np.random.default_rng(41).normal(size=(3, 64, 64))
    rng = np.random.default_rng(5)
    base = O.render(sc, cam, round_f32=False)
    vis = np.nonzero(base["proj"]["radius"] > 0)[0]
    picks = []
    for name in PARAMS:
        rows = sc[name].reshape(-1, sc["n"]).shape[0]
        for _ in range(24):
            picks.append((name, int(rng.integers(rows)) * sc["n"] + int(rng.choice(vis))))
    checked, skipped, _ = fd_check(sc, cam, w, picks)
    assert checked >= 0.8 * len(picks), (checked, skipped)


def test_single_gaussian_opacity_gradient_closed_form():
    # out = c a + (1 - a) bg with a = o G (unclamped, above 1/255):
    # dL/do = sum_p w_p . (c - bg) G_p ;  dL/dlogit = dL/do * o (1 - o)
    o = 0.6
    ls = -1.6
    W, H, f = 40, 36, 60.0
    bg = np.array([0.2, 0.5, 0.1])
    sh = np.zeros((1, 3, 1))
    sh[0, :, 0] = [0.8, -0.2, 0.4]
    sc = mk_scene([[0.0], [0.0], [0.0]], [ls], opacity_logits=[logit(o)], sh=sh)
    cam = axis_camera(W, H, f=f, bg=tuple(bg))
    w = np.random.default_rng(6).normal(size=(3, H, W))
    r = O.render(sc, cam, round_f32=False)
    g = O.backward(sc, cam, w, fwd=r, round_f32=False)
    var = (f32(f) * math.exp(f32(ls)) / 4.0) ** 2 + 0.3
    oo = 1.0 / (1.0 + math.exp(-f32(logit(o))))
    ys, xs = np.mgrid[0:H, 0:W]
    G = np.exp(-0.5 * ((xs - (W - 1) / 2) ** 2 + (ys - (H - 1) / 2) ** 2) / var)
    used = r["n_contrib"] > 0
    col = r["proj"]["rgb"][:, 0]
    bgf = bg.astype(np.float32).astype(np.float64)
    dLdo = float(((w * (col - bgf)[:, None, None]).sum(0) * G * used).sum())
    assert g["opacity_logits"][0] == pytest.approx(dLdo * oo * (1 - oo), rel=1e-12)


def test_l1_loss_gradient():
    img = np.array([[[0.2, 0.8]], [[0.5, 0.1]], [[0.9, 0.4]]])
    tgt = np.array([[[0.3, 0.7]], [[0.5, 0.2]], [[0.1, 0.4]]])
    g = O.l1_loss_grad(img, tgt)
    np.testing.assert_array_equal(g * 6, [[[-1, 1]], [[0, -1]], [[1, 0]]])
