"""Error paths of the C ABI on the GPU: an allocator that runs dry part way
through a render must give CDS_ERR_OOM and leave nothing allocated once the
frame and context are released; a corrupted tile list must be reported
through the device error word instead of being read out of bounds."""
import ctypes

import numpy as np
import pytest
import torch

from paper_2509_25626_amd import native
from paper_2509_25626_amd import scenes as S
from tests.conftest import gpu_available

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]


class LimitedAllocator:
    """Device allocator backed by torch tensors that refuses every request
    after the first `limit`; tracks what is still allocated."""

    def __init__(self, limit):
        self.limit = limit
        self.granted = 0
        self.live = {}
        self._a = native.CdsAllocator._fields_[0][1](self._alloc)
        self._f = native.CdsAllocator._fields_[1][1](self._free)
        self.struct = native.CdsAllocator(self._a, self._f, None)

    def _alloc(self, nbytes, _user):
        if self.granted >= self.limit:
            return None
        t = torch.empty(int(nbytes), dtype=torch.uint8, device="cuda")
        self.granted += 1
        self.live[t.data_ptr()] = t
        return t.data_ptr()

    def _free(self, ptr, _user):
        assert ptr in self.live, "free of a pointer the allocator never gave out"
        del self.live[ptr]


def _render_with_limit(L, limit, scene, cam, backward=False):
    from paper_2509_25626_amd.render import GaussianScene
    alloc = LimitedAllocator(limit)
    ctx = ctypes.c_void_p()
    st = L.cds_create(ctypes.byref(ctx), 0, ctypes.byref(alloc.struct))
    if st != native.CDS_OK:
        assert not ctx.value and not alloc.live
        alloc.message = L.cds_last_error()
        return st, None, alloc
    frame = ctypes.c_void_p()
    native.check(L.cds_frame_create(ctx, ctypes.byref(frame)))
    gs = GaussianScene.from_numpy(scene)
    sst = gs.struct()
    cs = native.camera_struct(cam)
    H, W = cam.height, cam.width
    rgb = torch.empty((3, H, W), device="cuda")
    T = torch.empty((H, W), device="cuda")
    nc = torch.empty((H, W), dtype=torch.int32, device="cuda")
    stream = torch.cuda.current_stream().cuda_stream
    st = L.cds_render_forward(ctx, frame, ctypes.byref(sst), ctypes.byref(cs), None, rgb.data_ptr(),
                              T.data_ptr(), nc.data_ptr(), stream)
    msg = L.cds_last_error() if st != native.CDS_OK else b""
    st_bwd = None
    if st == native.CDS_OK and backward:
        grads = {k: torch.empty_like(getattr(gs, k)) for k in
                 ("means", "log_scales", "quats", "opacity_logits", "sh")}
        g = native.CdsSceneGrad(*(grads[k].data_ptr() for k in
                                  ("means", "log_scales", "quats", "opacity_logits", "sh")))
        dl = torch.ones((3, H, W), device="cuda")
        st_bwd = L.cds_render_backward(ctx, frame, ctypes.byref(sst), ctypes.byref(cs), T.data_ptr(),
                                       nc.data_ptr(), dl.data_ptr(), ctypes.byref(g), stream)
    elif st != native.CDS_OK:
        # a failed forward leaves no render behind: backward and inspection refuse the frame
        fi = native.CdsFrameInfo()
        assert L.cds_frame_get_info(frame, ctypes.byref(fi)) == native.CDS_ERR_INVALID_ARG
    assert L.cds_check_device(ctx, stream) == native.CDS_OK
    L.cds_frame_release(frame)
    L.cds_destroy(ctx)
    torch.cuda.synchronize()
    alloc.message = msg
    return st, st_bwd, alloc


def test_allocator_exhaustion_reports_oom_without_leaks():
    L = native.load()
    scene = S.scene_outdoor(31, 20_000)
    cam = S.orbit_camera(200, 120, 4.0, 15.0, 5.0)
    results = []
    limit = 0
    while True:
        st, _, alloc = _render_with_limit(L, limit, scene, cam)
        assert not alloc.live, f"limit {limit}: {len(alloc.live)} allocations leaked"
        results.append(st)
        if st == native.CDS_OK:
            break
        assert st == native.CDS_ERR_OOM, (limit, native.STATUS_NAMES.get(st, st), getattr(alloc, "message", b""))
        assert limit == 0 or b"allocation" in alloc.message
        limit += 1
        assert limit < 200
    need = limit
    print(f"a forward render of this frame makes {need} device allocations; every smaller budget gave OOM")
    assert need > 10 and all(s == native.CDS_ERR_OOM for s in results[:-1])
    # backward needs more: with exactly the forward's budget it fails cleanly too
    st, st_bwd, alloc = _render_with_limit(L, need, scene, cam, backward=True)
    assert st == native.CDS_OK and st_bwd == native.CDS_ERR_OOM and not alloc.live
    st, st_bwd, alloc = _render_with_limit(L, need + 8, scene, cam, backward=True)
    assert st == native.CDS_OK and st_bwd == native.CDS_OK and not alloc.live


def test_corrupted_tile_list_sets_error_word():
    from paper_2509_25626_amd.render import GaussianScene, Renderer, _hip_runtime
    R = Renderer(0)
    try:
        scene = S.scene_outdoor(32, 5_000)
        cam = S.orbit_camera(96, 64, 4.0, 0.0, 0.0)
        gs = GaussianScene.from_numpy(scene)
        rgb, T, nc, frame = R.forward(gs, cam)
        torch.cuda.synchronize()
        R.check_device()
        fi = frame.info()
        rg = frame.fetch()["ranges"]
        ncn = nc.cpu().numpy()
        # the tile whose pixels blend the most splats: its first list entry is staged
        tiles_x = fi.tiles_x
        best, best_t = -1, -1
        for t in range(rg.shape[0]):
            ty, tx = divmod(t, tiles_x)
            m = int(ncn[ty * 16:(ty + 1) * 16, tx * 16:(tx + 1) * 16].max())
            if rg[t, 1] > rg[t, 0] and m > best:
                best, best_t = m, t
        assert best > 0
        bad = np.array([0xFFFFFFFF], np.uint32)
        pos = int(rg[best_t, 0])
        rc = _hip_runtime().hipMemcpy(fi.values + 4 * pos, bad.ctypes.data, 4, 1)  # host -> device
        assert rc == 0
        dl = torch.ones_like(rgb) / rgb.numel()
        R.backward(frame, gs, cam, T, nc, dl)
        with pytest.raises(native.CdsError) as e:
            R.check_device()
        assert e.value.status == native.CDS_ERR_DEVICE and "code 16" in str(e.value)
        R.check_device()  # the word was cleared by the report
        R.release_frame(frame)
    finally:
        R.close()
