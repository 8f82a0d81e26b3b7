"""Serving: resident scenes, continuous batching, admission by the HBM budget.

Each served image must be bit-identical to the single render of the same
scene and camera (so it is the same alone and in any mix of requests), and one
served image is checked against the CPU oracle directly.
"""
import numpy as np
import pytest
import torch

from paper_2509_25626_amd import scenes as S
from tests.conftest import gpu_available

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

RESOLUTIONS = [(640, 360), (333, 257), (97, 61), (256, 256), (1237, 822)]


@pytest.fixture(scope="module")
def resident():
    from paper_2509_25626_amd.render import GaussianScene
    sizes = [3_000, 20_000, 60_000, 150_000]
    np_scenes = [S.scene_outdoor(700 + k, n) for k, n in enumerate(sizes)]
    return np_scenes, [GaussianScene.from_numpy(s) for s in np_scenes]


@pytest.fixture(scope="module")
def R():
    from paper_2509_25626_amd.render import Renderer
    r = Renderer(0)
    yield r
    r.close()


def make_requests(seed, count, n_scenes):
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for _ in range(count):
        w, h = RESOLUTIONS[int(rng.integers(0, len(RESOLUTIONS)))]
        cam = S.orbit_camera(w, h, radius=4.0, azimuth_deg=float(rng.uniform(0, 360)),
                             elevation_deg=float(rng.uniform(-15, 15)))
        out.append((int(rng.integers(0, n_scenes)), cam))
    return out


def serve_all(srv, ids, reqs):
    outs = []
    tickets = []
    for sid, cam in reqs:
        t, o = srv.submit(ids[sid], cam)
        tickets.append(t)
        outs.append(o)
    srv.drain()
    for t in tickets:
        done, lat = srv.poll(t)
        assert done and lat >= 0
    torch.cuda.synchronize()
    return outs


def single_renders(R, scenes, reqs):
    out = []
    for sid, cam in reqs:
        rgb, _, _, frame = R.forward(scenes[sid], cam)
        out.append(rgb.clone())
        R.release_frame(frame)
    torch.cuda.synchronize()
    R.check_device()
    return out


@pytest.mark.parametrize("max_slots,max_batch,sort_variant", [(16, 8, 0), (1, 1, 0), (64, 64, 0), (16, 8, 2)])
def test_served_equals_single_render(R, resident, max_slots, max_batch, sort_variant):
    """Served images equal single renders bit for bit, with the batches' tile
    lists by row-wise placement over the stacked tile grid (default) or by
    radix-sorted stacked tile keys (sort variant 2)."""
    from paper_2509_25626_amd.serve import Server
    _, scenes = resident
    reqs = make_requests(11 + max_batch, 24, len(scenes))
    ref = single_renders(R, scenes, reqs)
    with Server(0, max_slots=max_slots, max_batch=max_batch, sort_variant=sort_variant) as srv:
        ids = [srv.add_scene(s) for s in scenes]
        got = serve_all(srv, ids, reqs)
        st = srv.stats()
    for k, (a, b) in enumerate(zip(got, ref)):
        assert torch.equal(a, b), f"request {k}: served image differs from the single render"
    assert st["submitted"] == len(reqs) and st["completed"] == len(reqs) and st["rejected"] == 0
    assert st["workspace_bytes"] == 0
    if max_batch == 1:
        assert st["batches"] == len(reqs)
    else:
        assert 1 <= st["batches"] <= len(reqs)


def test_same_request_alone_and_in_mix(R, resident):
    """One request served alone, then inside a mix of other scenes and
    resolutions submitted around it: identical bits."""
    from paper_2509_25626_amd.serve import Server
    _, scenes = resident
    probe = (2, S.orbit_camera(333, 257, azimuth_deg=40.0, elevation_deg=5.0))
    with Server(0, max_slots=16, max_batch=16) as srv:
        ids = [srv.add_scene(s) for s in scenes]
        alone = serve_all(srv, ids, [probe])[0].clone()
        mix = make_requests(5, 15, len(scenes))
        reqs = mix[:7] + [probe] + mix[7:]
        got = serve_all(srv, ids, reqs)
        st = srv.stats()
    assert torch.equal(got[7], alone)
    assert st["batches"] < st["submitted"], "no request was batched with another"


def test_served_image_matches_oracle(resident):
    from oracle import oracle as O
    from paper_2509_25626_amd.serve import Server
    from tests.test_gpu_parity import IMG_TOL, flip_mask
    np_scenes, scenes = resident
    cam = S.orbit_camera(97, 61, azimuth_deg=10.0)
    with Server(0, max_slots=4, max_batch=4) as srv:
        ids = [srv.add_scene(s) for s in scenes[:2]]
        reqs = [(1, S.orbit_camera(640, 360, azimuth_deg=200.0)), (0, cam), (1, cam)]
        got = serve_all(srv, ids, reqs)
    ora = O.render(np_scenes[0], cam)
    img = got[1].cpu().numpy().astype(np.float64)
    ok = ~flip_mask(ora)
    err = np.abs(img - ora["image"]).max(axis=0)
    assert err[ok].max() <= IMG_TOL
    assert (~ok).mean() < 0.01


def test_budget_rejects_oversized_request(resident):
    from paper_2509_25626_amd import native
    from paper_2509_25626_amd.serve import Server
    _, scenes = resident
    with Server(0, max_slots=4, max_batch=4, hbm_budget_bytes=1 << 20) as srv:
        big = srv.add_scene(scenes[3])
        small = srv.add_scene(scenes[0])
        with pytest.raises(native.CdsError) as ei:
            srv.submit(big, S.orbit_camera(1237, 822))
        assert ei.value.status == native.CDS_ERR_BUSY
        t, out = srv.submit(small, S.orbit_camera(97, 61))
        srv.drain()
        assert srv.poll(t)[0]
        st = srv.stats()
    assert st["rejected"] == 1 and st["completed"] == 1


def test_budget_binds_admission(R, resident):
    """A budget that holds about one large request: requests still all complete,
    with identical images, and neither the reserved workspace nor the device
    memory the workspaces' buffers actually hold ever exceeds the budget."""
    from paper_2509_25626_amd.serve import Server
    _, scenes = resident
    reqs = [(3, S.orbit_camera(640, 360, azimuth_deg=30.0 * k)) for k in range(6)]
    ref = single_renders(R, scenes, reqs)
    budget = 80 << 20
    with Server(0, max_slots=8, max_batch=8, hbm_budget_bytes=budget) as srv:
        ids = [srv.add_scene(s) for s in scenes]
        got = serve_all(srv, ids, reqs)
        st = srv.stats()
    for a, b in zip(got, ref):
        assert torch.equal(a, b)
    assert 0 < st["peak_workspace_bytes"] <= budget
    assert 0 < st["peak_held_bytes"] <= budget, st
    assert st["held_bytes"] <= budget
    assert st["batches"] >= 2


def test_invalid_requests(resident):
    from paper_2509_25626_amd import native
    from paper_2509_25626_amd.serve import Server
    _, scenes = resident
    with Server(0, max_slots=2, max_batch=2) as srv:
        sid = srv.add_scene(scenes[0])
        with pytest.raises(native.CdsError) as ei:
            srv.submit(sid + 5, S.orbit_camera(64, 64))
        assert ei.value.status == native.CDS_ERR_INVALID_ARG
        with pytest.raises(native.CdsError):
            srv.poll(12345)
    with pytest.raises(native.CdsError) as ei:
        Server(0, max_slots=2, max_batch=2, sort_variant=3)
    assert ei.value.status == native.CDS_ERR_INVALID_ARG
    with Server(0, max_slots=2, max_batch=2) as srv:
        sid = srv.add_scene(scenes[0])
        t, _ = srv.submit(sid, S.orbit_camera(64, 64))
        srv.drain()
        assert srv.poll(t)[0]
        with pytest.raises(native.CdsError):
            srv.poll(t)  # already collected
    with pytest.raises(native.CdsError):
        Server(0, max_slots=4, max_batch=8)
