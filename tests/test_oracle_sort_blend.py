"""Pins of the oracle's key/sort/range and blending stages (Sec. II-B, Eq. (1),
Algorithm 1) against brute force, invariants and closed forms."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2509_25626_amd import scenes as S
from tests.helpers import axis_camera, f32, logit, mk_scene

AMAX = float(np.float32(0.99))
AMIN = float(np.float32(1.0) / np.float32(255.0))
TMIN = float(np.float32(0.0001))


def _small_scene(n=600, W=70, H=45, seed=11, opacity_mu=0.0, deg=1):
    rng = np.random.Generator(np.random.PCG64(seed))
    means = rng.uniform(-1.5, 1.5, (3, n))
    sc = S.random_scene(rng, n, deg, means, -2.6, 0.6, opacity_mu, 1.5)
    cam = axis_camera(W, H, f=80.0, bg=(0.2, 0.3, 0.1))
    return sc, cam


# ------------------------------------------------------------------ keys / sort / ranges

def test_sort_matches_python_sorted():
    sc, cam = _small_scene(n=300)
    p = O.project(sc, cam)
    k, v = O.keys_unsorted(p, cam.width)
    ks, vs = O.sort_keys(k, v)
    # stable sort of (key, value) pairs generated in ascending index order
    ref = sorted(zip(k.tolist(), range(k.size)), key=lambda kv: kv[0])  # Python's sort is stable
    assert ks.tolist() == [a for a, _ in ref]
    assert vs.tolist() == [int(v[i]) for _, i in ref]


def test_keys_invariants_and_ranges():
    sc, cam = S.config_scene("c1")
    r = O.render(sc, cam)
    p, ks, vs, rg = r["proj"], r["keys"], r["vals"], r["ranges"]
    W, H = cam.width, cam.height
    tx, ty = O.tiles_xy(W, H)
    # permutation of the unsorted pairs
    assert np.array_equal(np.sort(r["keys_unsorted"]), ks)
    # within a tile: depth non-decreasing, equal depths by ascending index
    tile = (ks >> np.uint64(32)).astype(np.int64)
    depth = (ks & np.uint64(0xFFFFFFFF)).astype(np.int64)
    same = tile[1:] == tile[:-1]
    assert np.all(np.diff(tile) >= 0)
    assert np.all(depth[1:][same] >= depth[:-1][same])
    tie = same & (depth[1:] == depth[:-1])
    assert np.all(vs[1:][tie] > vs[:-1][tie])
    # per-tile counts from a 2D difference array over the rectangles
    diff = np.zeros((ty + 1, tx + 1), np.int64)
    vis = p["tiles_touched"] > 0
    x0, y0, x1, y1 = (p["rect"][i][vis] for i in range(4))
    np.add.at(diff, (y0, x0), 1)
    np.add.at(diff, (y0, x1 + 1), -1)
    np.add.at(diff, (y1 + 1, x0), -1)
    np.add.at(diff, (y1 + 1, x1 + 1), 1)
    counts = diff.cumsum(0).cumsum(1)[:ty, :tx].reshape(-1)
    assert np.array_equal(rg[:, 1] - rg[:, 0], counts)
    starts = np.concatenate([[0], np.cumsum(counts)[:-1]])
    nz = counts > 0
    assert np.array_equal(rg[nz, 0], starts[nz])
    assert np.all(rg[~nz] == 0)
    assert r["K"] == counts.sum()


# ------------------------------------------------------------------ blending

def test_single_isotropic_gaussian_closed_form():
    # One Gaussian on the axis: power = -d^2 / (2 var) with var = (f s / z)^2 + 0.3;
    # alpha = min(0.99, o e^power), kept when >= 1/255 inside the covered tiles.
    o = 0.7
    ls = -1.8
    W, H = 64, 48
    f = 120.0
    bg = (0.1, 0.2, 0.3)
    sh = np.zeros((1, 3, 1))
    sh[0, :, 0] = [0.4, -0.3, 1.1]
    sc = mk_scene([[0.0], [0.0], [0.0]], [ls], opacity_logits=[logit(o)], sh=sh)
    cam = axis_camera(W, H, f=f, bg=bg)
    r = O.render(sc, cam, round_f32=False)
    p = r["proj"]
    var = (f32(f) * math.exp(f32(ls)) / 4.0) ** 2 + 0.3
    oo = 1.0 / (1.0 + math.exp(-f32(logit(o))))
    col = np.maximum(sh[0, :, 0].astype(np.float32).astype(np.float64) / (2 * math.sqrt(math.pi)) + 0.5, 0)
    ys, xs = np.mgrid[0:H, 0:W]
    d2 = (xs - (W - 1) / 2) ** 2 + (ys - (H - 1) / 2) ** 2
    a = np.minimum(AMAX, oo * np.exp(-0.5 * d2 / var))
    tx0, ty0, tx1, ty1 = p["rect"][:, 0]
    inside = ((xs // 16 >= tx0) & (xs // 16 <= tx1) & (ys // 16 >= ty0) & (ys // 16 <= ty1))
    a = np.where((a >= AMIN) & inside, a, 0.0)
    bgv = np.array([f32(b) for b in bg])
    expect = a[None] * col[:, None, None] + (1 - a)[None] * bgv[:, None, None]
    np.testing.assert_allclose(r["image"], expect, rtol=0, atol=1e-12)
    np.testing.assert_allclose(r["final_T"], 1 - a, atol=1e-14)
    assert np.array_equal(r["n_contrib"], (a > 0).astype(np.uint32))


def _two_stack(depth_a, depth_b, o=0.9, bg=(0.0, 0.0, 0.0)):
    sh = np.zeros((1, 3, 2))
    sh[0, :, 0] = [2.0, -2.0, -2.0]   # reddish
    sh[0, :, 1] = [-2.0, 2.0, -2.0]   # greenish
    sc = mk_scene(np.array([[0.0, 0.0], [0.0, 0.0], [depth_a, depth_b]]), [-1.0, -1.0],
                  opacity_logits=[logit(o), logit(o)], sh=sh)
    cam = axis_camera(33, 33, f=50.0, bg=bg)
    r = O.render(sc, cam, round_f32=False)
    return r, r["proj"]


def test_two_opaque_gaussians_occlude_in_depth_order():
    # Centre pixel, G = 1 for both: out = near*0.9 + far*0.9*0.1 + bg*0.01.
    bg = (0.25, 0.5, 0.75)
    r, p = _two_stack(-0.5, 0.5, bg=bg)
    o = 1.0 / (1.0 + math.exp(-f32(logit(0.9))))
    c = 16
    near, far = p["rgb"][:, 0], p["rgb"][:, 1]
    bgv = np.array([f32(b) for b in bg])
    np.testing.assert_allclose(r["image"][:, c, c], near * o + far * o * (1 - o) + bgv * (1 - o) ** 2,
                               atol=1e-12)
    assert r["n_contrib"][c, c] == 2
    r2, p2 = _two_stack(0.5, -0.5, bg=bg)   # swap the depths: colours swap
    np.testing.assert_allclose(r2["image"][:, c, c], far * o + near * o * (1 - o) + bgv * (1 - o) ** 2,
                               atol=1e-12)


def test_alpha_clamp_and_termination_with_float32_constants():
    # Two clamped (alpha = 0.99f) Gaussians: T' = (1-0.99f)^2 = 9.99998e-5 < 1e-4f,
    # so the second one is not blended (the threshold test comes before accumulation).
    r, p = _two_stack(-0.5, 0.5, o=0.9999)
    c = 16
    near = p["rgb"][:, 0]
    np.testing.assert_allclose(r["image"][:, c, c], near * AMAX, atol=1e-12)
    assert r["n_contrib"][c, c] == 1
    assert r["final_T"][c, c] == pytest.approx(1 - AMAX, abs=1e-15)
    assert (1 - AMAX) ** 2 < TMIN
    # the stopping Gaussian is examined but not blended: two entries examined
    assert r["n_eval"][c, c] == 2


def test_examined_entries_count():
    # Per pixel, the entries the front-to-back walk examines (Alg. 1): through
    # the one whose T(1 - alpha) falls below 1e-4, else the whole tile list.
    # Single pass over two stacked half-opaque Gaussians: never stops, so every
    # pixel examines its tile's whole list.
    r, _ = _two_stack(-0.5, 0.5, o=0.5)
    lens = (r["ranges"][:, 1] - r["ranges"][:, 0]).astype(np.int64)
    W = r["image"].shape[2]
    tiles_x = (W + 15) // 16
    ys, xs = np.mgrid[0:r["image"].shape[1], 0:W]
    per_pixel_len = lens[(ys // 16) * tiles_x + xs // 16]
    assert np.array_equal(r["n_eval"], per_pixel_len)
    # A random scene: examined >= last blended position, <= the list length,
    # and a pixel that stopped early examined exactly one entry past the last
    # one it blended or skipped before stopping, so n_eval > n_contrib there.
    sc, cam = _small_scene(n=800, opacity_mu=3.0)
    r = O.render(sc, cam, round_f32=True)
    lens = (r["ranges"][:, 1] - r["ranges"][:, 0]).astype(np.int64)
    tiles_x = (cam.width + 15) // 16
    ys, xs = np.mgrid[0:cam.height, 0:cam.width]
    L = lens[(ys // 16) * tiles_x + xs // 16]
    ne, nc = r["n_eval"].astype(np.int64), r["n_contrib"].astype(np.int64)
    assert np.all(ne >= nc) and np.all(ne <= L)
    stopped = ne < L
    assert stopped.any() and np.all(ne[stopped] > nc[stopped])
    # where the walk ran to the end of the list, T never fell below 1e-4 by blending
    assert np.all(r["final_T"][~stopped] >= TMIN)


def test_eq1_three_layer_composite():
    # C = sum_i T_i a_i c_i with T_i = prod_{j<i} (1 - a_j), out = C + T bg  (Eq. (1), splat alpha)
    ops = [0.6, 0.5, 0.8]
    sh = np.zeros((1, 3, 3))
    sh[0] = np.array([[1.0, -0.5, 0.2], [0.3, 0.9, -1.0], [-0.2, 0.4, 0.7]])
    sc = mk_scene(np.array([[0.0, 0.0, 0.0], [0.0, 0.0, 0.0], [0.8, -0.6, 0.1]]), [-1.0] * 3,
                  opacity_logits=[logit(o) for o in ops], sh=sh)
    bg = (0.3, 0.6, 0.9)
    r = O.render(sc, axis_camera(33, 33, f=50.0, bg=bg), round_f32=False)
    p = r["proj"]
    order = np.argsort(p["depth"])
    T = 1.0
    C = np.zeros(3)
    for i in order:
        a = p["opacity"][i]
        C += T * a * p["rgb"][:, i]
        T *= 1 - a
    C += T * np.array([f32(b) for b in bg])
    np.testing.assert_allclose(r["image"][:, 16, 16], C, atol=1e-12)
    assert r["n_contrib"][16, 16] == 3


@pytest.mark.parametrize("round_f32", [True, False])
def test_tile_path_equals_brute_force(round_f32):
    sc, cam = _small_scene(n=500)
    r = O.render(sc, cam, round_f32=round_f32)
    img, T, nc, margins, used = O.blend_brute(r["proj"], cam, tile_filter=True)
    assert np.array_equal(img, r["image"])
    assert np.array_equal(T, r["final_T"])
    assert np.array_equal(nc, r["n_contrib"])
    assert np.array_equal(used, r["n_used"])
    assert (nc > 0).mean() > 0.5


def test_lossless_tile_culling_when_opacity_below_bound():
    # With every o < e^4.5 / 255 ~= 0.353 no pixel outside the 3-sigma square reaches
    # alpha >= 1/255, so dropping the rectangle filter changes nothing.
    sc, cam = _small_scene(n=500, opacity_mu=-2.5)
    sc["opacity_logits"] = np.minimum(sc["opacity_logits"], np.float32(logit(0.35)))
    r = O.render(sc, cam)
    img, T, nc, _, used = O.blend_brute(r["proj"], cam, tile_filter=False)
    assert np.array_equal(img, r["image"])
    assert np.array_equal(T, r["final_T"])
    # n_contrib is a list position (skipped entries count), so only the number of
    # Gaussians actually blended is list-independent
    assert np.array_equal(used, r["n_used"])


def test_rect_filter_is_lossy_for_opaque_gaussians():
    # Counter-check of the bound above: with high opacities some alpha >= 1/255 lies
    # outside the covered square, so the unfiltered brute force differs somewhere.
    sc, cam = _small_scene(n=500, opacity_mu=4.0)
    r = O.render(sc, cam)
    img, _, _, _, _ = O.blend_brute(r["proj"], cam, tile_filter=False)
    assert not np.array_equal(img, r["image"])


def test_c1_statistics_and_margins():
    sc, cam = S.config_scene("c1")
    r = O.render(sc, cam)
    assert 35_000 < r["K"] < 46_000
    flip = O.flip_eligible_pixels(r["margins"], r["n_used"])
    assert flip.mean() < 2e-4
    assert r["image"].min() >= 0.0
