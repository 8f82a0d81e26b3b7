"""Pins of the oracle's projection and colour stages (Sec. II-B(1); 3DGS EWA
projection) against closed forms, library routines and brute force."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from tests.helpers import axis_camera, mk_scene, f32

F = 200.0
W, H = 96, 80


def _cam():
    cam = axis_camera(W, H, f=F)
    return cam


@pytest.mark.parametrize("ls", [-3.0, -2.0, -1.2])
@pytest.mark.parametrize("quat", [(1, 0, 0, 0), (0.3, -0.5, 0.7, 0.2), (-2.0, 1.0, 0.5, -0.1)])
def test_isotropic_on_axis_closed_form(ls, quat):
    # An isotropic Gaussian on the optical axis at depth 4: Sigma' = ((f s / z)^2 + 0.3) I,
    # whatever its rotation; the larger "eigenvalue" used for the radius is
    # sigma'^2 + sqrt(0.1) because the discriminant is floored at 0.1.
    sc = mk_scene([[0.0], [0.0], [0.0]], [ls], quats=np.array(quat, float).reshape(4, 1))
    p = O.project(sc, _cam(), round_f32=False)
    s = math.exp(f32(ls))
    f = f32(F)
    var = (f * s / 4.0) ** 2 + 0.3
    assert p["radius"][0] == math.ceil(3.0 * math.sqrt(var + math.sqrt(0.1)))
    np.testing.assert_allclose(p["conic"][:, 0], [1.0 / var, 0.0, 1.0 / var], rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(p["mean2d"][:, 0], [(W - 1) / 2, (H - 1) / 2], rtol=0, atol=1e-12)
    assert p["depth_bits"][0] == np.float32(4.0).view(np.uint32)


@pytest.mark.parametrize("xyz", [(0.5, -0.3, 1.0), (-1.1, 0.9, -0.5), (0.0, 1.2, 2.0), (0.2, 0.1, -2.5)])
def test_isotropic_off_axis_jacobian_closed_form(xyz):
    # R = I camera, isotropic Sigma = s^2 I: Sigma' = s^2 J J^T + 0.3 I with
    # J = (f/z)[[1, 0, -x/z], [0, 1, -y/z]]  =>  J J^T = (f/z)^2 [[1+u^2, uv], [uv, 1+v^2]].
    ls = -2.0
    sc = mk_scene(np.array(xyz).reshape(3, 1), [ls])
    p = O.project(sc, _cam(), round_f32=False)
    x, y, z = (f32(c) for c in xyz)
    z += 4.0
    u, v = x / z, y / z
    f = f32(F)
    # the Jacobian's ratios are limited to 1.3x the half field of view
    limx, limy = 1.3 * W / (2 * f), 1.3 * H / (2 * f)
    uc, vc = min(max(u, -limx), limx), min(max(v, -limy), limy)
    s2 = math.exp(2 * f32(ls))
    k = s2 * (f / z) ** 2
    a, b, c = k * (1 + uc * uc) + 0.3, k * uc * vc, k * (1 + vc * vc) + 0.3
    inv = np.linalg.inv(np.array([[a, b], [b, c]]))
    np.testing.assert_allclose(p["conic"][:, 0], [inv[0, 0], inv[0, 1], inv[1, 1]], rtol=1e-11)
    np.testing.assert_allclose(p["mean2d"][:, 0], [f * u + (W - 1) / 2, f * v + (H - 1) / 2], rtol=1e-13)


def test_guard_band_clamp_closed_form():
    # x/z beyond 1.3 * W / (2 f): the Jacobian uses the clamped ratio, the mean does not.
    ls = -2.0
    limx = 1.3 * W / (2 * f32(F))
    z = 4.0
    x = f32(1.6 * limx * z)
    y = f32(0.05 * z)
    sc = mk_scene(np.array([x, y, 0.0]).reshape(3, 1), [ls])
    p = O.project(sc, _cam(), round_f32=False)
    u, v = limx, y / z
    s2 = math.exp(2 * f32(ls))
    k = s2 * (f32(F) / z) ** 2
    a, b, c = k * (1 + u * u) + 0.3, k * u * v, k * (1 + v * v) + 0.3
    inv = np.linalg.inv(np.array([[a, b], [b, c]]))
    if p["radius"][0] > 0:  # may be off-screen; the conic is defined either way when visible
        np.testing.assert_allclose(p["conic"][:, 0], [inv[0, 0], inv[0, 1], inv[1, 1]], rtol=1e-11)
    assert p["clamp_flags"][0] & O.CF_JX


def test_rotation_convention_quarter_turn_about_z():
    # A quarter turn about z maps the x axis to y: scales (sx, sy) rotated equal (sy, sx) unrotated.
    pos = np.array([[0.3], [-0.2], [0.4]])
    h = math.sqrt(0.5)
    a = mk_scene(pos, np.array([[-1.5], [-2.5], [-2.0]]), quats=np.array([[h], [0], [0], [h]]))
    b = mk_scene(pos, np.array([[-2.5], [-1.5], [-2.0]]))
    pa = O.project(a, _cam(), round_f32=False)
    pb = O.project(b, _cam(), round_f32=False)
    np.testing.assert_allclose(pa["conic"], pb["conic"], rtol=1e-6)
    assert pa["radius"][0] == pb["radius"][0]


def test_quaternion_scale_and_sign_invariance():
    rng = np.random.default_rng(3)
    n = 64
    means = rng.uniform(-1, 1, (3, n))
    ls = rng.normal(-2.5, 0.4, (3, n))
    q = rng.normal(size=(4, n))
    p0 = O.project(mk_scene(means, ls, quats=q), _cam(), round_f32=False)
    for scale in (-1.0, 3.5):
        p1 = O.project(mk_scene(means, ls, quats=scale * q), _cam(), round_f32=False)
        # float32 storage of the scaled quaternion changes the last bits only
        np.testing.assert_allclose(p1["conic"], p0["conic"], rtol=1e-5, atol=1e-9)


def test_rotation_matrix_orthonormal_via_isotropic_invariance():
    # Sigma = R s^2 R^T equals s^2 I only if R(q) is orthonormal for every unit q.
    rng = np.random.default_rng(4)
    n = 200
    means = np.zeros((3, n))
    q = rng.normal(size=(4, n))
    ref = O.project(mk_scene(means, np.full((3, n), -2.0)), _cam(), round_f32=False)
    rot = O.project(mk_scene(means, np.full((3, n), -2.0), quats=q), _cam(), round_f32=False)
    np.testing.assert_allclose(rot["conic"], ref["conic"], rtol=1e-12, atol=1e-14)


def test_radius_matches_eigen_decomposition():
    rng = np.random.default_rng(5)
    n = 300
    means = rng.uniform(-1.2, 1.2, (3, n))
    ls = rng.normal(-2.0, 0.8, (3, n))
    q = rng.normal(size=(4, n))
    p = O.project(mk_scene(means, ls, quats=q), _cam(), round_f32=False)
    checked = 0
    for i in range(n):
        if p["radius"][i] == 0 or p["near_flags"][i] & O.NF_RADIUS:
            continue
        A, B, C = p["conic"][:, i]
        cov = np.linalg.inv(np.array([[A, B], [B, C]]))
        lo, hi = np.linalg.eigvalsh(cov)
        mid = 0.5 * (lo + hi)
        lam = mid + math.sqrt(max(0.1, (0.5 * (hi - lo)) ** 2))
        assert p["radius"][i] == math.ceil(3.0 * math.sqrt(lam)), i
        checked += 1
    assert checked > 100


def test_near_plane_cull():
    sc = mk_scene(np.array([[0.0, 0.0], [0.0, 0.0], [-3.81, -3.79]]), [-3.0, -3.0])
    p = O.project(sc, _cam(), round_f32=False)
    assert p["radius"][0] == 0 and p["tiles_touched"][0] == 0  # t_z = 0.19
    assert p["radius"][1] > 0 and p["tiles_touched"][1] > 0    # t_z = 0.21


def test_tile_rect_brute_force():
    # Covered tiles = tiles holding a pixel p with |p - mean|_inf <= r (mean as stored, float32).
    rng = np.random.default_rng(6)
    n = 400
    Wi, Hi = 50, 37
    cam = axis_camera(Wi, Hi, f=60.0)
    means = np.stack([rng.uniform(-3, 3, n), rng.uniform(-3, 3, n), rng.uniform(-2, 2, n)])
    ls = rng.normal(-2.5, 0.7, (3, n))
    p = O.project(mk_scene(means, ls, quats=rng.normal(size=(4, n))), cam, round_f32=True)
    ys, xs = np.mgrid[0:Hi, 0:Wi]
    vis = 0
    for i in range(n):
        r = p["radius"][i]
        mx, my = p["mean2d"][:, i]
        if r == 0:  # culled: behind the near plane or no pixel within r
            continue
        cover = (np.abs(xs - mx) <= r) & (np.abs(ys - my) <= r)
        assert cover.any()
        tys, txs = np.nonzero(cover)
        tset = set(zip((txs // 16).tolist(), (tys // 16).tolist()))
        tx0, ty0, tx1, ty1 = p["rect"][:, i]
        rect = {(tx, ty) for tx in range(tx0, tx1 + 1) for ty in range(ty0, ty1 + 1)}
        assert rect == tset, i
        assert p["tiles_touched"][i] == len(rect)
        vis += 1
    assert vis > 100


def test_depth_bits_are_float32_of_view_depth():
    rng = np.random.default_rng(7)
    n = 100
    means = rng.uniform(-1, 1, (3, n))
    p = O.project(mk_scene(means, np.full((3, n), -3.0)), _cam(), round_f32=True)
    z = means[2].astype(np.float32).astype(np.float64) + 4.0
    vis = p["radius"] > 0
    assert np.array_equal(p["depth_bits"][vis], z[vis].astype(np.float32).view(np.uint32))
    # positive float32 bit patterns order like the values
    order_bits = np.argsort(p["depth_bits"][vis], kind="stable")
    order_vals = np.argsort(z[vis].astype(np.float32), kind="stable")
    assert np.array_equal(order_bits, order_vals)


def test_depth_tie_rounds_to_even_and_is_not_flagged():
    # A view depth exactly on a float32 rounding midpoint (4 + 2^-22 lies
    # halfway between 4 and the next float32 above it) is an exact tie: IEEE
    # round-to-nearest-even takes 4.0 in any implementation that computes the
    # same double, so it is not ambiguous and carries no flag.  A depth a
    # hair above the midpoint (2^-45, a 6e-8 ulp margin) is ambiguous between
    # evaluation orders and is flagged; it rounds up.
    tie = np.float32(2.0 ** -22)
    above = np.nextafter(tie, np.float32(1.0))
    sc = mk_scene(np.array([[0.0, 0.0], [0.0, 0.0], [tie, above]]), [-3.0, -3.0])
    p = O.project(sc, _cam(), round_f32=True)
    assert p["depth"][0] == 4.0 + 2.0 ** -22 and p["depth"][1] > p["depth"][0]
    assert p["depth_bits"][0] == np.float32(4.0).view(np.uint32)
    assert p["depth_bits"][1] == np.nextafter(np.float32(4.0), np.float32(5.0)).view(np.uint32)
    assert p["near_flags"][0] & O.NF_DEPTH_ROUND == 0
    assert p["near_flags"][1] & O.NF_DEPTH_ROUND != 0


def test_colour_on_axis_closed_form():
    # Straight ahead of an R = I camera the view direction is (0, 0, 1): only the
    # m = 0 harmonics survive, Y_00 = 1/(2 sqrt(pi)), Y_10 = sqrt(3/(4 pi)) z,
    # Y_20 = sqrt(5/(16 pi)) (2z^2 - x^2 - y^2), Y_30 = sqrt(7/(16 pi)) z (2z^2 - 3x^2 - 3y^2).
    rng = np.random.default_rng(8)
    sh = rng.normal(0, 0.3, (16, 3, 1))
    sh[0] = rng.uniform(0, 1, (3, 1))
    sc = mk_scene([[0.0], [0.0], [0.5]], [-2.0], sh=sh, sh_degree=3)
    p = O.project(sc, _cam(), round_f32=False)
    s = sh.astype(np.float32).astype(np.float64)[:, :, 0]
    pi = math.pi
    raw = (s[0] / (2 * math.sqrt(pi)) + math.sqrt(3 / (4 * pi)) * s[2]
           + math.sqrt(5 / (16 * pi)) * 2 * s[6] + math.sqrt(7 / (16 * pi)) * 2 * s[12] + 0.5)
    np.testing.assert_allclose(p["rgb"][:, 0], np.maximum(raw, 0.0), rtol=1e-12, atol=1e-14)


def test_colour_clamped_at_zero():
    sh = np.zeros((1, 3, 1))
    sh[0, :, 0] = [-5.0, 0.0, 5.0]
    p = O.project(mk_scene([[0.0], [0.0], [0.0]], [-2.0], sh=sh), _cam(), round_f32=False)
    assert p["rgb"][0, 0] == 0.0 and p["clamp_flags"][0] & O.CF_R
    assert p["rgb"][1, 0] == pytest.approx(0.5)


def test_sh_basis_orthonormal_by_quadrature():
    # Gauss-Legendre in cos(theta) x uniform in phi integrates degree <= 6 products exactly.
    nt, nphi = 16, 32
    xg, wg = np.polynomial.legendre.leggauss(nt)
    phi = 2 * np.pi * np.arange(nphi) / nphi
    ct, ph = np.meshgrid(xg, phi, indexing="ij")
    st = np.sqrt(1 - ct ** 2)
    dirs = np.stack([st * np.cos(ph), st * np.sin(ph), ct], -1).reshape(-1, 3)
    w = (np.repeat(wg, nphi) * (2 * np.pi / nphi))
    Y = O.sh_basis(dirs, 3)
    G = (Y * w[:, None]).T @ Y
    np.testing.assert_allclose(G, np.eye(16), atol=1e-12)


def test_sh_basis_matches_scipy_real_combination():
    # Real harmonics from scipy's complex ones (which carry the Condon-Shortley
    # phase): m > 0 -> sqrt(2) Re Y_l^m, m < 0 -> sqrt(2) Im Y_l^|m|, m = 0 -> Y_l^0.
    sp = pytest.importorskip("scipy.special")
    rng = np.random.default_rng(9)
    d = rng.normal(size=(50, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    theta = np.arccos(d[:, 2])           # polar
    phi = np.arctan2(d[:, 1], d[:, 0])   # azimuth
    Y = O.sh_basis(d, 3)
    col = 0
    for l in range(4):
        for m in range(-l, l + 1):
            am = abs(m)
            if hasattr(sp, "sph_harm_y"):
                c = sp.sph_harm_y(l, am, theta, phi)
            else:
                c = sp.sph_harm(am, l, phi, theta)
            ref = c.real if m == 0 else (math.sqrt(2) * c.real if m > 0 else math.sqrt(2) * c.imag)
            np.testing.assert_allclose(Y[:, col], ref, atol=1e-12, err_msg=f"l={l} m={m}")
            col += 1


def test_sh_band_energy_rotation_invariant():
    # Rotating the direction mixes coefficients within a band only.
    rng = np.random.default_rng(10)
    d = rng.normal(size=(3000, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    Y0 = O.sh_basis(d, 3)
    Y1 = O.sh_basis(d @ q.T, 3)
    for lo, hi in ((0, 1), (1, 4), (4, 9), (9, 16)):
        np.testing.assert_allclose((Y0[:, lo:hi] ** 2).sum(1), (Y1[:, lo:hi] ** 2).sum(1), atol=1e-12)
