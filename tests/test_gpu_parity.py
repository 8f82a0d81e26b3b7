"""GPU parity of the HIP path against the CPU oracle, through the C ABI.

Per stage: projection (radius, rectangle, tiles touched and depth bits
bit-exact; mean, conic, opacity, colour within float32 rounding), keys, values
and tile ranges bit-exact, images within 1e-5 absolute per channel except at
pixels where a blending decision sits within float32 rounding of its
threshold (counted, must stay rare), n_contrib exact elsewhere.
"""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2509_25626_amd import scenes as S
from tests.conftest import gpu_available
from tests.helpers import axis_camera, mk_scene

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

IMG_TOL = 1e-5


@pytest.fixture(scope="module")
def R():
    from paper_2509_25626_amd.render import Renderer
    r = Renderer(0)
    yield r
    r.close()


def gpu_render(R, scene, cam, variant=0, sort_variant=0, sort_algo="auto"):
    from paper_2509_25626_amd.render import GaussianScene
    gs = GaussianScene.from_numpy(scene)
    rgb, T, nc, frame = R.forward(gs, cam, blend_variant=variant, sort_variant=sort_variant,
                                  sort_algo=sort_algo)
    torch.cuda.synchronize()
    R.check_device()
    out = dict(image=rgb.cpu().numpy(), final_T=T.cpu().numpy(),
               n_contrib=nc.cpu().numpy().view(np.uint32))
    out.update(frame.fetch())
    R.release_frame(frame)
    return out


def unpack_rect(tr):
    return np.stack([tr[:, 0] & 0xFFFF, tr[:, 0] >> 16, tr[:, 1] & 0xFFFF, tr[:, 1] >> 16]).astype(np.int32)


def flip_mask(ora):
    """Pixels where float32 and float64 may legitimately take different blending branches."""
    return O.flip_eligible_pixels(ora["margins"], ora["n_used"])


def compare_projection(g, o):
    """Per-Gaussian projection.  Returns the Gaussians whose discrete outputs
    the oracle flags as within rounding of a decision boundary; their GPU
    values are checked to be one of the legitimate alternatives here and are
    reconciled with the oracle's key list by `reconcile_flagged`."""
    p = o["proj"]
    flagged = (p["near_flags"] & O.NF_KEY_DECISIONS) != 0
    ok = ~flagged
    assert np.array_equal(g["radius"][ok], p["radius"][ok])
    assert np.array_equal(g["tiles_touched"][ok], p["tiles_touched"][ok])
    assert np.array_equal(g["depth_bits"][ok], p["depth_bits"][ok])
    vis = ok & (p["radius"] > 0)
    assert np.array_equal(unpack_rect(g["tile_rect"])[:, vis], p["rect"][:, vis])
    # float32 values of float64 results: within two ulps
    np.testing.assert_allclose(g["mean2d"][vis].T, p["mean2d"][:, vis], rtol=2.5e-7, atol=1e-6)
    np.testing.assert_allclose(g["conic_opacity"][vis, :3].T, p["conic"][:, vis], rtol=1e-6, atol=1e-9)
    np.testing.assert_allclose(g["conic_opacity"][vis, 3], p["opacity"][vis], rtol=2.5e-7, atol=1e-9)
    # colour: float32 SH evaluation
    np.testing.assert_allclose(g["rgb"][vis, :3].T, p["rgb"][:, vis], rtol=0, atol=2e-6)
    # flagged: the GPU took one of the two roundings the oracle's margin allows
    both = flagged & (p["radius"] > 0) & (g["radius"] > 0)
    if both.any():
        assert np.abs(g["radius"][both].astype(np.int64) - p["radius"][both]).max() <= 1
        assert np.abs(g["depth_bits"][both].astype(np.int64) - p["depth_bits"][both].astype(np.int64)).max() <= 1
        np.testing.assert_allclose(g["mean2d"][both].T, p["mean2d"][:, both], rtol=2.5e-7, atol=1e-6)
        d = np.abs(unpack_rect(g["tile_rect"])[:, both] - p["rect"][:, both])
        assert d.max() <= 1
    return flagged


def reconcile_flagged(g, o, flagged, cam):
    """Oracle result to compare against when flagged Gaussians exist.

    A flagged Gaussian's radius, 2D mean, rectangle or depth bits sit within
    rounding of a boundary, so either neighbouring value is correct.  Where
    the GPU took the other one, the oracle's values for that Gaussian are
    replaced by the GPU's and the oracle's own key build, sort, ranges and
    blend run again; everything is then compared in full.  Returns the
    (possibly recomputed) oracle result and the number of Gaussians replaced.
    """
    if not flagged.any():
        return o, 0
    p = o["proj"]
    rect_g = unpack_rect(g["tile_rect"])
    vis_g = g["radius"] > 0
    diff = flagged & ((g["radius"] != p["radius"]) | (g["depth_bits"] != p["depth_bits"])
                      | (g["tiles_touched"] != p["tiles_touched"])
                      | np.any(np.where(vis_g, rect_g, 0) != p["rect"], axis=0)
                      | np.any(g["mean2d"].T.astype(np.float64) != p["mean2d"], axis=0))
    idx = np.nonzero(diff)[0]
    if idx.size == 0:
        return o, 0
    q = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in p.items()}
    q["radius"][idx] = g["radius"][idx]
    q["tiles_touched"][idx] = g["tiles_touched"][idx]
    q["depth_bits"][idx] = g["depth_bits"][idx]
    q["rect"][:, idx] = np.where(vis_g[idx], rect_g[:, idx], 0)
    q["mean2d"][:, idx] = g["mean2d"][idx].T.astype(np.float64)
    # a Gaussian only the GPU keeps visible blends with the GPU's float32 values
    only_g = idx[(p["radius"][idx] == 0) & vis_g[idx]]
    q["conic"][:, only_g] = g["conic_opacity"][only_g, :3].T
    q["opacity"][only_g] = g["conic_opacity"][only_g, 3]
    q["rgb"][:, only_g] = g["rgb"][only_g, :3].T
    W, H = cam.width, cam.height
    k0, v0 = O.keys_unsorted(q, W)
    ks, vs = O.sort_keys(k0, v0)
    rg = O.ranges(ks, W, H)
    img, T, nc, margins, used = O.blend_tiles(q, rg, vs, cam)
    o2 = dict(o, proj=q, keys_unsorted=k0, vals_unsorted=v0, keys=ks, vals=vs, ranges=rg,
              image=img, final_T=T, n_contrib=nc, margins=margins, n_used=used, K=int(ks.size))
    return o2, int(idx.size)


def effective_sort_variant(sort_variant):
    """The variant a render runs (the default is row-wise placement; every
    image the tests render is within its 4096 tiles per axis)."""
    return 4 if sort_variant == 0 else sort_variant


def expected_offsets(o, sort_variant):
    sort_variant = effective_sort_variant(sort_variant)
    if sort_variant in (3, 4):  # binning and row-wise placement never form the key offsets
        return np.zeros(0, np.uint32)
    t = o["proj"]["tiles_touched"].astype(np.uint64)
    if sort_variant == 2:  # visible splats visited in (depth bits, index) order
        vis = np.nonzero(t > 0)[0]
        t = t[vis[np.argsort(o["proj"]["depth_bits"][vis], kind="stable")]]
    return np.concatenate([[0], np.cumsum(t)[:-1]]).astype(np.uint32) if t.size else np.zeros(0, np.uint32)


def compare_keys(g, o, sort_variant=0):
    """K, key offsets, every sorted key and value, and every tile range,
    bit-exact against the oracle (Sec. II-B(1) duplication and sort, Alg. 1
    ranges).  `o` is the oracle result after `reconcile_flagged`."""
    assert g["K"] == o["K"]
    assert np.array_equal(g["tiles_touched"], o["proj"]["tiles_touched"])
    vis = o["proj"]["radius"] > 0
    assert np.array_equal(unpack_rect(g["tile_rect"])[:, vis], o["proj"]["rect"][:, vis])
    assert np.array_equal(g["offsets"], expected_offsets(o, sort_variant))
    assert np.array_equal(g["keys"], o["keys"])
    assert np.array_equal(g["values"], o["vals"])
    assert np.array_equal(g["ranges"], o["ranges"])


def compare_images(g, o, max_flip_frac=1e-3):
    flip = flip_mask(o)
    good = ~flip
    assert flip.mean() <= max_flip_frac, flip.mean()
    err = np.abs(g["image"] - o["image"]).max(axis=0)
    assert err[good].max() <= IMG_TOL, (err[good].max(), np.unravel_index(np.argmax(np.where(good, err, 0)), err.shape))
    assert np.abs(g["final_T"] - o["final_T"])[good].max() <= IMG_TOL
    assert np.array_equal(g["n_contrib"][good], o["n_contrib"][good])
    return int(flip.sum())


def full_check(R, scene, cam, variant=0, sort_variant=0, sort_algo="auto"):
    g = gpu_render(R, scene, cam, variant, sort_variant, sort_algo)
    o = O.render(scene, cam, round_f32=True)
    flagged = compare_projection(g, o)
    o, _ = reconcile_flagged(g, o, flagged, cam)
    compare_keys(g, o, sort_variant)
    nflip = compare_images(g, o)
    return g, o, nflip


# ---------------------------------------------------------------- whole pipeline

@pytest.mark.parametrize("sort_variant,sort_algo", [(0, "auto"), (1, "auto"), (2, "auto"), (3, "auto"), (4, "auto"),
                                                     (2, "onesweep"), (2, "reduce_scan"), (1, "reduce_scan"),
                                                     (3, "reduce_scan")])
def test_c1_forward_parity(R, sort_variant, sort_algo):
    scene, cam = S.config_scene("c1")
    g, o, nflip = full_check(R, scene, cam, sort_variant=sort_variant, sort_algo=sort_algo)
    # 40 key bits: 5 radix passes, 4 of them over the depth digits when presorted
    assert g["K"] > 30000 and g["passes"] == (4 if effective_sort_variant(sort_variant) in (3, 4) else 5)
    print(f"c1: K={g['K']} flip-eligible pixels={nflip}")


@pytest.mark.parametrize("wh,n", [((203, 117), 30_000), ((16, 16), 30_000), ((1, 1), 30_000),
                                  ((1237, 822), 40_000), ((8192, 300), 20_000), ((5000, 64), 9_000),
                                  ((2200, 2000), 30_000)])
def test_sort_variants_bit_identical(R, wh, n):
    # every digit per key == depth digits per Gaussian + tile digits per key ==
    # depth digits per Gaussian + tile binning.  The wide images give bands of
    # fewer than 16 tile rows and (8192x300) longer chunks for a large tile grid;
    # 2200x2000 has more tiles (17,250) than one LDS difference array holds, so
    # its tile counts go through record chunks.
    W, H = wh
    scene = S.scene_outdoor(15, n)
    cam = S.orbit_camera(W, H, 4.0, 10.0, 0.0)
    a = gpu_render(R, scene, cam, sort_variant=1)
    for sv in (2, 3, 4):
        b = gpu_render(R, scene, cam, sort_variant=sv)
        for k in ("keys", "values", "ranges", "image", "final_T", "n_contrib"):
            # offsets: the visit order differs by design (index order vs depth order)
            assert np.array_equal(a[k], b[k]), (sv, k)
        assert a["K"] == b["K"]


def test_binning_many_keys_per_row(R):
    # large splats: a (chunk, tile row) holds far more keys than one placement
    # pass stages, so rows are placed in several passes over tile ranges
    scene = S.scene_outdoor(16, 12_000, log_scale_mu=-1.2, log_scale_sigma=0.3)
    cam = S.orbit_camera(1237, 822, 4.0, 30.0, 0.0)
    a = gpu_render(R, scene, cam, sort_variant=1)
    assert a["K"] > 12_000 * 100
    for sv in (3, 4):
        b = gpu_render(R, scene, cam, sort_variant=sv)
        for k in ("keys", "values", "ranges", "image", "final_T", "n_contrib"):
            assert np.array_equal(a[k], b[k]), (sv, k)


@pytest.mark.parametrize("variant", [1, 2])
def test_blend_cull_long_thin_splats(R, variant):
    # splats hundreds of pixels long and under a pixel thin at every angle,
    # many centred far from the tiles they cross, with opacities down to
    # 1/255: the per-row-group ellipse test of the staged splats sits at the
    # edge of its margin here (large offsets, steep forms); the image must
    # still match the oracle and the two pixel layouts agree bit for bit
    rng = np.random.Generator(np.random.PCG64(31))
    n = 4000
    scene = S.scene_c1(32, n)
    ls = np.empty((3, n))
    ls[0] = rng.normal(0.3, 0.4, size=n)    # long axis
    ls[1] = rng.normal(-6.5, 0.3, size=n)   # thin
    ls[2] = rng.normal(-6.5, 0.3, size=n)
    scene["log_scales"] = ls.astype(np.float32)
    logit = np.log((1.0 / 255.0) / (1.0 - 1.0 / 255.0))
    op = rng.normal(0.0, 2.0, size=n)
    op[: n // 4] = rng.normal(logit, 0.05, size=n // 4)
    scene["opacity_logits"] = op.astype(np.float32)
    cam = S.orbit_camera(333, 257, 3.5, 35.0, 10.0)
    g = gpu_render(R, scene, cam, variant)
    o = O.render(scene, cam, round_f32=True)
    compare_images(g, o, max_flip_frac=5e-3)
    other = gpu_render(R, scene, cam, 3 - variant)
    for k in ("image", "final_T", "n_contrib"):
        assert np.array_equal(g[k], other[k]), k


@pytest.mark.parametrize("variant", [1, 2, 3, 4])
def test_blend_cull_edge_splats(R, variant):
    # the blend visits a splat only where its alpha can reach 1/255: opacities
    # straddling 1/255 and needle-thin, rotated splats sit right at the edge
    # of that region; the image must still match the oracle, and the three
    # pixel layouts (different per-wave regions) must agree bit for bit
    rng = np.random.Generator(np.random.PCG64(23))
    n = 6000
    scene = S.scene_c1(24, n)
    logit = np.log((1.0 / 255.0) / (1.0 - 1.0 / 255.0))
    op = rng.normal(logit, 0.05, size=n)
    op[: n // 3] = rng.normal(0.5, 1.5, size=n // 3)
    scene["opacity_logits"] = op.astype(np.float32)
    ls = rng.normal(-3.5, 0.5, size=(3, n))
    thin = rng.random(n) < 0.5
    ls[0, thin] = rng.normal(-1.5, 0.3, size=thin.sum())  # long axis
    ls[1, thin] = rng.normal(-6.5, 0.3, size=thin.sum())  # needle-thin
    scene["log_scales"] = ls.astype(np.float32)
    cam = S.orbit_camera(203, 117, 3.0, 20.0, 15.0)
    g = gpu_render(R, scene, cam, variant)
    o = O.render(scene, cam, round_f32=True)
    compare_images(g, o, max_flip_frac=5e-3)
    base = gpu_render(R, scene, cam, 2)
    for k in ("image", "final_T", "n_contrib"):
        assert np.array_equal(g[k], base[k]), k


@pytest.mark.parametrize("mu,sigma,n", [(-7.0, 0.3, 200_000), (-4.5, 2.0, 100_000), (-1.0, 0.2, 3_000)])
def test_generated_keys_match_duplication(R, mu, sigma, n):
    # the first tile pass generates the keys from the depth-ordered splat
    # records; with tiny splats (about one tile each) most 1024-key chunks
    # start more records than the generator's window holds, so it takes its
    # round-by-round path; wide size mixes alternate both paths, and large
    # splats span many chunks.  Reference: keys duplicated by their own kernel
    # (reduce-then-scan passes) and the 64-bit key sort.
    scene = S.scene_outdoor(18, n, log_scale_mu=mu, log_scale_sigma=sigma)
    cam = S.orbit_camera(1237, 822, 4.0, 30.0, 0.0)
    a = gpu_render(R, scene, cam, sort_variant=1)
    for sv, algo in ((2, "onesweep"), (2, "reduce_scan"), (4, "auto")):
        b = gpu_render(R, scene, cam, sort_variant=sv, sort_algo=algo)
        assert a["K"] == b["K"]
        for k in ("keys", "values", "ranges", "image", "final_T", "n_contrib"):
            assert np.array_equal(a[k], b[k]), (sv, algo, k)
    if mu < -6:  # under 4 keys per record: more than 256 records start in most chunks
        assert a["K"] < 3 * b["n_vis"]


@pytest.mark.parametrize("variant", [1, 2, 3, 4, 5])
def test_blend_variants_bit_identical(R, variant):
    scene, cam = S.config_scene("c1")
    base = gpu_render(R, scene, cam, 2)
    g = gpu_render(R, scene, cam, variant)
    assert np.array_equal(g["image"], base["image"])
    assert np.array_equal(g["final_T"], base["final_T"])
    assert np.array_equal(g["n_contrib"], base["n_contrib"])


def test_forward_deterministic(R):
    scene, cam = S.config_scene("c1")
    a = gpu_render(R, scene, cam)
    b = gpu_render(R, scene, cam)
    for k in ("image", "final_T", "n_contrib", "keys", "values", "ranges"):
        assert np.array_equal(a[k], b[k]), k


def test_frames_in_flight_on_two_streams(R):
    """Renders into two frames on two streams, each enqueued while the other
    is still running, give the same bits as the same renders one at a time."""
    from paper_2509_25626_amd.render import GaussianScene
    scene = GaussianScene.from_numpy(S.scene_outdoor(91, 150_000))
    cams = [S.orbit_camera(640, 360, azimuth_deg=37.0 * k, elevation_deg=4.0 * k - 6.0) for k in range(4)]
    ref = []
    frame = R.acquire_frame()
    for cam in cams:
        rgb, T, nc, _ = R.forward(scene, cam, frame=frame)
        ref.append((rgb.clone(), T.clone(), nc.clone()))
    R.release_frame(frame)
    torch.cuda.synchronize()
    frames = [R.acquire_frame(), R.acquire_frame()]
    streams = [torch.cuda.current_stream(), torch.cuda.Stream()]
    # each frame first renders every camera on its own stream, so its buffers
    # reach their size there (a buffer grown on a stream other than the one it
    # was allocated on would go back to the other stream's pool)
    for f, st in zip(frames, streams):
        with torch.cuda.stream(st):
            for cam in cams:
                R.forward(scene, cam, frame=f)
    torch.cuda.synchronize()
    got = []
    for i in range(12):
        with torch.cuda.stream(streams[i % 2]):
            rgb, T, nc, _ = R.forward(scene, cams[i % 4], frame=frames[i % 2])
            got.append((i % 4, rgb, T, nc))
    torch.cuda.synchronize()
    for f in frames:
        R.release_frame(f)
    R.check_device()
    for k, rgb, T, nc in got:
        assert torch.equal(rgb, ref[k][0]) and torch.equal(T, ref[k][1]) and torch.equal(nc, ref[k][2]), k
    # the renderer's own sequence helper, three renders in flight
    outs = R.forward_sequence(scene, cams * 2, in_flight=3)
    torch.cuda.synchronize()
    R.check_device()
    assert len(outs) == 2 * len(cams)
    for i, (rgb, T, nc) in enumerate(outs):
        k = i % len(cams)
        assert torch.equal(rgb, ref[k][0]) and torch.equal(T, ref[k][1]) and torch.equal(nc, ref[k][2]), i


def test_outdoor_sh3_ragged_image(R):
    # the outdoor distribution (ball + far shell, SH degree 3) shrunk to 20k Gaussians,
    # a 203 x 117 image (ragged 16x16 tiles) seen from an orbit pose with a coloured background
    scene = S.scene_outdoor(12, 20_000)
    cam = S.orbit_camera(203, 117, 4.0, 35.0, 10.0, bg=(0.2, 0.4, 0.6))
    g, o, nflip = full_check(R, scene, cam)
    assert g["K"] > 1000


def test_camera_inside_scene_near_plane(R):
    # camera inside the Gaussian ball: huge near-plane splats covering many tiles
    scene = S.scene_outdoor(13, 15_000, ball_radius=5.0)
    cam = S.orbit_camera(160, 96, 4.0, 0.0, 0.0)
    full_check(R, scene, cam)


def test_empty_and_fully_culled_scenes(R):
    cam = axis_camera(37, 23, f=40.0, bg=(0.3, 0.2, 0.1))
    empty = mk_scene(np.zeros((3, 0)), np.zeros((3, 0)), quats=np.zeros((4, 0)),
                     opacity_logits=np.zeros(0), sh=np.zeros((1, 3, 0)))
    behind = mk_scene(np.array([[0.0, 0.1], [0.0, 0.2], [-5.0, -6.0]]), [-2.0, -2.0])
    for sc in (empty, behind):
        g = gpu_render(R, sc, cam)
        assert g["K"] == 0
        bg = np.array(cam.bg, np.float32)[:, None, None]
        assert np.array_equal(g["image"], np.broadcast_to(bg, g["image"].shape))
        assert np.all(g["final_T"] == 1.0) and np.all(g["n_contrib"] == 0)


@pytest.mark.parametrize("wh", [(1, 1), (16, 16), (17, 3), (33, 65)])
def test_small_and_ragged_images(R, wh):
    W, H = wh
    rng = np.random.default_rng(W * 100 + H)
    n = 300
    means = rng.uniform(-1, 1, (3, n))
    sc = S.random_scene(rng, n, 1, means, -2.0, 0.5, 0.5, 1.5)
    cam = axis_camera(W, H, f=max(W, H) * 0.9)
    full_check(R, sc, cam)


def test_single_gaussian_covering_whole_image(R):
    sc = mk_scene([[0.0], [0.0], [0.0]], [0.3], opacity_logits=[2.0])
    cam = axis_camera(250, 130, f=150.0)
    g, o, _ = full_check(R, sc, cam)
    assert g["tiles_touched"][0] == 16 * 9


# ---------------------------------------------------------------- sort and scan

SORT_CASES = ([(c, b, "auto") for c in (1, 100, 4095, 4096, 4097, 123_457, 1_000_003) for b in (64, 44, 8)]
              + [(c, b, a) for c in (1, 4097, 1_000_003, 9_000_001) for b in (64, 12)
                 for a in ("onesweep", "reduce_scan")])


@pytest.mark.parametrize("count,end_bit,algo", SORT_CASES)
def test_sort_pairs_matches_stable_argsort(R, count, end_bit, algo):
    rng = np.random.default_rng(count + end_bit)
    # few distinct values so that ties (and therefore stability) matter
    keys = rng.integers(0, 2**63, size=count, dtype=np.uint64) & np.uint64(0xFFFF0000000F00FF)
    keys[rng.random(count) < 0.3] = np.uint64(7)
    vals = np.arange(count, dtype=np.uint32)
    kt = torch.from_numpy(keys.view(np.int64)).cuda()
    vt = torch.from_numpy(vals.view(np.int32)).cuda()
    ko, vo = R.sort_pairs(kt, vt, end_bit, algo)
    R.check_device()
    mask = np.uint64((1 << end_bit) - 1) if end_bit < 64 else np.uint64(0xFFFFFFFFFFFFFFFF)
    order = np.argsort(keys & mask, kind="stable")
    assert np.array_equal(ko.cpu().numpy().view(np.uint64), keys[order])
    assert np.array_equal(vo.cpu().numpy().view(np.uint32), vals[order])


@pytest.mark.parametrize("count", [0, 1, 4095, 4097, 1_000_003])
def test_exclusive_scan(R, count):
    rng = np.random.default_rng(count)
    v = rng.integers(0, 300, size=count, dtype=np.uint32)
    vt = torch.from_numpy(v.view(np.int32)).cuda()
    out, total = R.exclusive_scan(vt)
    ref = np.concatenate([[0], np.cumsum(v, dtype=np.uint64)[:-1]]) if count else np.zeros(0, np.uint64)
    assert np.array_equal(out.cpu().numpy().view(np.uint32), ref.astype(np.uint32))
    assert int(total.item()) == int(v.astype(np.uint64).sum())


# ---------------------------------------------------------------- backward

def _grad_check(R, scene, cam, seed, for_backward=False):
    from paper_2509_25626_amd.render import GaussianScene
    H, W = cam.height, cam.width
    dl = np.random.default_rng(seed).normal(size=(3, H, W)).astype(np.float32)
    gs = GaussianScene.from_numpy(scene)
    rgb, T, nc, frame = R.forward(gs, cam, for_backward=for_backward)
    grads = R.backward(frame, gs, cam, T, nc, torch.from_numpy(dl).cuda())
    torch.cuda.synchronize()
    R.release_frame(frame)
    o = O.render(scene, cam, round_f32=True)
    og = O.backward(scene, cam, dl.astype(np.float64), fwd=o, round_f32=True)
    report = {}
    for k in ("means", "log_scales", "quats", "opacity_logits", "sh"):
        gg = grads[k].cpu().numpy().astype(np.float64).reshape(-1)
        oo = og[k].reshape(-1)
        rel = np.linalg.norm(gg - oo) / max(np.linalg.norm(oo), 1e-30)
        elem_ok = np.abs(gg - oo) <= 1e-3 * np.abs(oo) + 1e-6 * np.abs(oo).max()
        report[k] = (rel, elem_ok.mean())
        assert rel <= 1e-4, (k, rel)
        assert elem_ok.mean() >= 0.999, (k, elem_ok.mean())
    return report


# for_backward: the forward keeps the colour's direction derivative and the
# backward reads it instead of the SH coefficients (SH degree > 0)
@pytest.mark.parametrize("for_backward", [False, True])
def test_backward_matches_oracle_gradients(R, for_backward):
    scene = S.scene_fd_subcase(41, 500)
    cam = S.orbit_camera(64, 64, 4.0, 20.0, 5.0, bg=(0.1, 0.2, 0.3))
    print(_grad_check(R, scene, cam, 1, for_backward))


@pytest.mark.parametrize("for_backward", [False, True])
def test_backward_outdoor_ragged(R, for_backward):
    scene = S.scene_outdoor(14, 4000)
    cam = S.orbit_camera(120, 72, 4.0, 60.0, -8.0, bg=(0.5, 0.5, 0.5))
    print(_grad_check(R, scene, cam, 2, for_backward))


@pytest.mark.parametrize("deg", [1, 2])
def test_backward_low_sh_degrees(R, deg):
    """SH degrees 1 and 2, with and without the kept colour derivative."""
    scene = S.scene_outdoor(15 + deg, 2000)
    nb = (deg + 1) ** 2
    scene = dict(scene, sh=np.ascontiguousarray(scene["sh"][:nb]), sh_degree=deg)
    cam = S.orbit_camera(96, 80, 4.0, 110.0, 12.0, bg=(0.2, 0.1, 0.0))
    for fb in (False, True):
        print(deg, fb, _grad_check(R, scene, cam, 3 + deg, fb))


def test_l1_loss_grad_kernel(R):
    rng = np.random.default_rng(3)
    a = rng.random((3, 20, 30)).astype(np.float32)
    b = rng.random((3, 20, 30)).astype(np.float32)
    a[0, 0, 0] = b[0, 0, 0]
    g, loss = R.l1_loss_grad(torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda())
    assert np.array_equal(g.cpu().numpy(), (np.sign(a - b) / a.size).astype(np.float32))
    assert loss.item() == pytest.approx(np.abs(a - b).mean(), rel=1e-5)


def test_autograd_function(R):
    from paper_2509_25626_amd.render import RenderFn
    scene = S.scene_fd_subcase(41, 300)
    cam = S.orbit_camera(48, 40, 4.0, 0.0, 0.0)
    ts = {k: torch.from_numpy(np.ascontiguousarray(scene[k])).cuda().requires_grad_(True)
          for k in ("means", "log_scales", "quats", "opacity_logits", "sh")}
    img = RenderFn.apply(R, cam, ts["means"], ts["log_scales"], ts["quats"], ts["opacity_logits"], ts["sh"])
    tgt = torch.rand_like(img)
    (img - tgt).abs().mean().backward()
    for k, t in ts.items():
        assert t.grad is not None and torch.isfinite(t.grad).all(), k
    assert ts["opacity_logits"].grad.abs().sum() > 0


def test_invalid_arguments_rejected(R):
    from paper_2509_25626_amd import native
    from paper_2509_25626_amd.render import GaussianScene
    scene = S.scene_fd_subcase(41, 50)
    gs = GaussianScene.from_numpy(scene)
    cam = S.orbit_camera(32, 32)
    bad = S.orbit_camera(32, 32)
    bad.width = 0
    with pytest.raises(native.CdsError) as e:
        R.forward(gs, bad)
    assert e.value.status == native.CDS_ERR_INVALID_ARG
    with pytest.raises(native.CdsError):
        R.forward(gs, cam, blend_variant=6)
    bad = S.orbit_camera(32, 32)
    bad.near_plane = 0.0
    with pytest.raises(native.CdsError):
        R.forward(gs, bad)
