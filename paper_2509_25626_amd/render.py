"""PyTorch-facing API of the renderer: scenes as device tensors, a renderer
context, forward/backward calls, and an autograd Function.

PyTorch provides device memory (through an allocator callback) and streams
(the current stream is passed to every call); all arithmetic runs in the
library's HIP kernels.
"""
from __future__ import annotations

import ctypes
import weakref

import numpy as np
import torch

from . import native
from .native import P, check

__all__ = ["GaussianScene", "Renderer", "RenderFn", "render", "device_to_numpy"]

_hip = None


def _hip_runtime():
    global _hip
    if _hip is None:
        _hip = ctypes.CDLL("libamdhip64.so")
        _hip.hipMemcpy.argtypes = [P, P, ctypes.c_size_t, ctypes.c_int]
        _hip.hipMemcpy.restype = ctypes.c_int
    return _hip


def device_to_numpy(ptr: int, count: int, dtype) -> np.ndarray:
    """Copy `count` elements at a device address into a new numpy array."""
    out = np.empty(int(count), dtype=dtype)
    if count:
        torch.cuda.synchronize()
        rc = _hip_runtime().hipMemcpy(out.ctypes.data, ptr, out.nbytes, 2)  # device -> host
        if rc != 0:
            raise RuntimeError(f"hipMemcpy failed with {rc}")
    return out


def _sort_flag(algo: str) -> int:
    return {"auto": 0, "onesweep": native.CDS_OPT_SORT_ONESWEEP,
            "reduce_scan": native.CDS_OPT_SORT_REDUCE_SCAN}[algo]


def _stream_handle(device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


class _TorchAllocator:
    """Device allocator callback backed by torch tensors (torch owns the memory)."""

    def __init__(self, device):
        self.device = device
        self.blocks = {}
        self._alloc_cb = native.CdsAllocator._fields_[0][1](self._alloc)
        self._free_cb = native.CdsAllocator._fields_[1][1](self._free)
        self.struct = native.CdsAllocator(self._alloc_cb, self._free_cb, None)

    def _alloc(self, nbytes, _user):
        try:
            t = torch.empty(int(nbytes), dtype=torch.uint8, device=self.device)
        except torch.OutOfMemoryError:
            return None
        ptr = t.data_ptr()
        self.blocks[ptr] = t
        return ptr

    def _free(self, ptr, _user):
        self.blocks.pop(ptr, None)


class GaussianScene:
    """N Gaussians as float32 structure-of-arrays device tensors:
    means [3,N], log_scales [3,N], quats [4,N] (w,x,y,z), opacity_logits [N],
    sh [(deg+1)^2, 3, N]."""

    def __init__(self, means, log_scales, quats, opacity_logits, sh, sh_degree=None):
        self.means = means.contiguous()
        self.log_scales = log_scales.contiguous()
        self.quats = quats.contiguous()
        self.opacity_logits = opacity_logits.contiguous()
        self.sh = sh.contiguous()
        n = self.means.shape[-1]
        k = self.sh.shape[0]
        deg = int(round(k ** 0.5)) - 1 if sh_degree is None else int(sh_degree)
        if (deg + 1) ** 2 != k:
            raise ValueError("sh must have (deg+1)^2 coefficient planes")
        for name, t, shape in (("means", self.means, (3, n)), ("log_scales", self.log_scales, (3, n)),
                               ("quats", self.quats, (4, n)), ("opacity_logits", self.opacity_logits, (n,)),
                               ("sh", self.sh, (k, 3, n))):
            if tuple(t.shape) != shape or t.dtype != torch.float32 or not t.is_cuda:
                raise ValueError(f"{name} must be a float32 CUDA tensor of shape {shape}")
        self.n = n
        self.sh_degree = deg

    @classmethod
    def from_numpy(cls, scene: dict, device="cuda"):
        t = lambda k: torch.as_tensor(np.ascontiguousarray(scene[k], dtype=np.float32), device=device)
        return cls(t("means"), t("log_scales"), t("quats"), t("opacity_logits"), t("sh"),
                   scene["sh_degree"])

    def struct(self) -> native.CdsScene:
        s = native.CdsScene()
        s.n = self.n
        s.sh_degree = self.sh_degree
        s.means = self.means.data_ptr()
        s.log_scales = self.log_scales.data_ptr()
        s.quats = self.quats.data_ptr()
        s.opacity_logits = self.opacity_logits.data_ptr()
        s.sh = self.sh.data_ptr()
        return s

    def nbytes(self) -> int:
        return sum(t.numel() * 4 for t in (self.means, self.log_scales, self.quats,
                                           self.opacity_logits, self.sh))


class Frame:
    def __init__(self, renderer, handle):
        self.renderer = renderer
        self.handle = handle

    def info(self) -> native.CdsFrameInfo:
        fi = native.CdsFrameInfo()
        check(native.load().cds_frame_get_info(self.handle, ctypes.byref(fi)))
        return fi

    def stage_times(self) -> dict:
        st = native.CdsStageTimes()
        check(native.load().cds_frame_stage_times(self.handle, ctypes.byref(st)))
        return {k: float(getattr(st, k)) for k, _ in native.CdsStageTimes._fields_}

    def release(self):
        if self.handle:
            native.load().cds_frame_release(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.release()
        except Exception:
            pass

    def fetch(self) -> dict:
        """Copy the frame's per-stage state to host numpy arrays (for tests)."""
        fi = self.info()
        n, K = fi.n, fi.num_keys
        ntiles = fi.tiles_x * fi.tiles_y
        g = lambda ptr, cnt, dt: device_to_numpy(ptr, cnt, dt) if ptr else np.zeros(0, dt)
        noff = fi.num_visible if fi.offsets and fi.num_visible != n else n
        return dict(
            n=n, K=K, tiles_x=fi.tiles_x, tiles_y=fi.tiles_y, passes=fi.sort_passes, n_vis=fi.num_visible,
            mean2d=g(fi.mean2d, 2 * n, np.float32).reshape(n, 2),
            conic_opacity=g(fi.conic_opacity, 4 * n, np.float32).reshape(n, 4),
            rgb=g(fi.rgb, 4 * n, np.float32).reshape(n, 4),
            depth_bits=g(fi.depth_bits, n, np.uint32), radius=g(fi.radius, n, np.int32),
            tile_rect=g(fi.tile_rect, 2 * n, np.uint32).reshape(n, 2),
            tiles_touched=g(fi.tiles_touched, n, np.uint32), offsets=g(fi.offsets, noff, np.uint32),
            keys=g(fi.keys, K, np.uint64), values=g(fi.values, K, np.uint32),
            ranges=g(fi.ranges, 2 * ntiles, np.uint32).reshape(ntiles, 2),
            clamp_flags=g(fi.clamp_flags, n, np.uint8))


class Renderer:
    """A library context on one device, with a pool of frames.

    Renders run on the current torch stream.  Renders into different frames
    may be in flight on different streams at once; keep each frame on one
    stream (or synchronise before moving it): its buffers come from torch's
    allocator on the stream that was current when they were allocated, and
    one that grows is handed back to that stream's pool."""

    def __init__(self, device: int = 0, torch_allocator: bool = True):
        self.L = native.load()
        self.device = torch.device("cuda", device)
        self._alloc = _TorchAllocator(self.device) if torch_allocator else None
        h = P()
        check(self.L.cds_create(ctypes.byref(h), device,
                                ctypes.byref(self._alloc.struct) if self._alloc else None))
        self.handle = h
        self._pool = []
        self._frames = weakref.WeakSet()

    def close(self):
        if self.handle:
            torch.cuda.synchronize(self.device)  # no render still uses a frame's buffers
        for f in list(self._frames):
            f.release()
        self._pool = []
        self._seq = None
        if self.handle:
            self.L.cds_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def acquire_frame(self) -> Frame:
        if self._pool:
            return self._pool.pop()
        h = P()
        check(self.L.cds_frame_create(self.handle, ctypes.byref(h)))
        f = Frame(self, h)
        self._frames.add(f)
        return f

    def release_frame(self, frame: Frame):
        self._pool.append(frame)

    def forward_sequence(self, scene: GaussianScene, cams, in_flight: int = 2, **kw):
        """Render `cams` in order with `in_flight` renders overlapping, each on
        a stream and frame of its own (kept by the renderer for later calls);
        returns [(rgb, final_T, n_contrib)] in camera order, ready for work on
        the caller's current stream.  `kw` as for forward (no frame or out)."""
        if in_flight < 1:
            raise ValueError("in_flight must be at least 1")
        seq = getattr(self, "_seq", None)
        if seq is None or len(seq) != in_flight:
            if seq is not None:
                torch.cuda.synchronize(self.device)  # the old streams' renders are done
                for f, _ in seq:
                    f.release()
            seq = []
            for _ in range(in_flight):
                h = P()
                check(self.L.cds_frame_create(self.handle, ctypes.byref(h)))
                f = Frame(self, h)
                self._frames.add(f)
                seq.append((f, torch.cuda.Stream(self.device)))
            self._seq = seq
        cur = torch.cuda.current_stream(self.device)
        for _, st in seq:
            st.wait_stream(cur)  # the scene and earlier work on the caller's stream
        outs = []
        for i, cam in enumerate(cams):
            f, st = seq[i % in_flight]
            with torch.cuda.stream(st):
                rgb, T, nc, _ = self.forward(scene, cam, frame=f, **kw)
            for t in (rgb, T, nc):
                t.record_stream(cur)
            outs.append((rgb, T, nc))
        for _, st in seq:
            cur.wait_stream(st)
        return outs

    def forward(self, scene: GaussianScene, cam, frame: Frame | None = None, blend_variant: int = 0,
                out=None, timing: bool = False, sort_variant: int = 0, sort_algo: str = "auto",
                invdepth=None, for_backward: bool = False):
        """Render; returns (rgb [3,H,W], final_T [H,W], n_contrib [H,W] int32 view of uint32, frame).
        With `invdepth` (True, or an [H,W] float32 tensor to fill) the expected
        inverse depth is rendered too and returned as a fifth element.
        `for_backward`: the render will be differentiated (CDS_OPT_KEEP_FOR_BACKWARD:
        the frame keeps the colour's direction derivative for the backward pass)."""
        cs = native.camera_struct(cam)
        H, W = cs.height, cs.width
        if out is None:
            rgb = torch.empty((3, H, W), dtype=torch.float32, device=self.device)
            T = torch.empty((H, W), dtype=torch.float32, device=self.device)
            nc = torch.empty((H, W), dtype=torch.int32, device=self.device)
        else:
            rgb, T, nc = out
        frame = frame or self.acquire_frame()
        flags = ((native.CDS_OPT_STAGE_TIMING if timing else 0) | _sort_flag(sort_algo) |
                 (native.CDS_OPT_KEEP_FOR_BACKWARD if for_backward else 0))
        opts = native.CdsRenderOpts(flags, int(blend_variant), int(sort_variant), 0)
        sst = scene.struct()
        if invdepth is None:
            check(self.L.cds_render_forward(self.handle, frame.handle, ctypes.byref(sst), ctypes.byref(cs),
                                            ctypes.byref(opts), rgb.data_ptr(), T.data_ptr(), nc.data_ptr(),
                                            _stream_handle(self.device)))
            return rgb, T, nc, frame
        if invdepth is True:
            invdepth = torch.empty((H, W), dtype=torch.float32, device=self.device)
        check(self.L.cds_render_forward_ex(self.handle, frame.handle, ctypes.byref(sst), ctypes.byref(cs),
                                           ctypes.byref(opts), rgb.data_ptr(), T.data_ptr(), nc.data_ptr(),
                                           invdepth.data_ptr(), _stream_handle(self.device)))
        return rgb, T, nc, frame, invdepth

    def backward(self, frame: Frame, scene: GaussianScene, cam, T, nc, dL_drgb, grads=None, dL_dinvdepth=None):
        """Gradients of the last forward render of `frame` (and of its inverse
        depth, with `dL_dinvdepth` [H,W]); returns a dict of tensors."""
        cs = native.camera_struct(cam)
        if grads is None:
            grads = {k: torch.empty_like(getattr(scene, k))
                     for k in ("means", "log_scales", "quats", "opacity_logits", "sh")}
        g = native.CdsSceneGrad(*(grads[k].data_ptr() for k in
                                  ("means", "log_scales", "quats", "opacity_logits", "sh")))
        dl = dL_drgb.contiguous()
        sst = scene.struct()
        if dL_dinvdepth is None:
            check(self.L.cds_render_backward(self.handle, frame.handle, ctypes.byref(sst), ctypes.byref(cs),
                                             T.data_ptr(), nc.data_ptr(), dl.data_ptr(), ctypes.byref(g),
                                             _stream_handle(self.device)))
        else:
            dd = dL_dinvdepth.contiguous()
            check(self.L.cds_render_backward_ex(self.handle, frame.handle, ctypes.byref(sst), ctypes.byref(cs),
                                                T.data_ptr(), nc.data_ptr(), dl.data_ptr(), dd.data_ptr(),
                                                ctypes.byref(g), _stream_handle(self.device)))
        return grads

    def l1_loss_grad(self, rgb, target, grad=None, loss=None):
        grad = torch.empty_like(rgb) if grad is None else grad
        loss = torch.empty(1, dtype=torch.float32, device=self.device) if loss is None else loss
        check(self.L.cds_l1_loss_grad(self.handle, rgb.data_ptr(), target.data_ptr(), rgb.numel(),
                                      grad.data_ptr(), loss.data_ptr(), _stream_handle(self.device)))
        return grad, loss

    def sort_pairs(self, keys, values, end_bit=64, algo="auto"):
        """Stable radix sort of uint64 keys (int64 tensor bits) with uint32 values (int32 bits)."""
        ko = torch.empty_like(keys)
        vo = torch.empty_like(values)
        check(self.L.cds_sort_pairs(self.handle, keys.data_ptr(), values.data_ptr(), keys.numel(),
                                    int(end_bit), ko.data_ptr(), vo.data_ptr(), _sort_flag(algo),
                                    _stream_handle(self.device)))
        return ko, vo

    def exclusive_scan(self, values):
        out = torch.empty_like(values)
        total = torch.empty(1, dtype=torch.int64, device=self.device)
        check(self.L.cds_exclusive_scan_u32(self.handle, values.data_ptr(), values.numel(), out.data_ptr(),
                                            total.data_ptr(), _stream_handle(self.device)))
        return out, total

    def check_device(self):
        check(self.L.cds_check_device(self.handle, _stream_handle(self.device)))


class RenderFn(torch.autograd.Function):
    """Differentiable render: image = RenderFn.apply(renderer, cam, means, log_scales, quats,
    opacity_logits, sh).  Backward runs the library's adjoint kernels."""

    @staticmethod
    def forward(ctx, renderer, cam, means, log_scales, quats, opacity_logits, sh):
        scene = GaussianScene(means.detach(), log_scales.detach(), quats.detach(),
                              opacity_logits.detach(), sh.detach())
        rgb, T, nc, frame = renderer.forward(scene, cam, for_backward=True)
        ctx.renderer, ctx.cam, ctx.scene, ctx.frame = renderer, cam, scene, frame
        ctx.save_for_backward(T, nc)
        return rgb

    @staticmethod
    def backward(ctx, grad_rgb):
        T, nc = ctx.saved_tensors
        g = ctx.renderer.backward(ctx.frame, ctx.scene, ctx.cam, T, nc, grad_rgb)
        ctx.renderer.release_frame(ctx.frame)
        ctx.frame = None
        return (None, None, g["means"], g["log_scales"], g["quats"], g["opacity_logits"], g["sh"])


class RenderDepthFn(torch.autograd.Function):
    """Differentiable render with the expected inverse depth: (image, invdepth) =
    RenderDepthFn.apply(renderer, cam, means, log_scales, quats, opacity_logits, sh)."""

    @staticmethod
    def forward(ctx, renderer, cam, means, log_scales, quats, opacity_logits, sh):
        scene = GaussianScene(means.detach(), log_scales.detach(), quats.detach(),
                              opacity_logits.detach(), sh.detach())
        rgb, T, nc, frame, invd = renderer.forward(scene, cam, invdepth=True, for_backward=True)
        ctx.renderer, ctx.cam, ctx.scene, ctx.frame = renderer, cam, scene, frame
        ctx.save_for_backward(T, nc)
        return rgb, invd

    @staticmethod
    def backward(ctx, grad_rgb, grad_invdepth):
        T, nc = ctx.saved_tensors
        if grad_rgb is None:
            grad_rgb = torch.zeros((3,) + tuple(T.shape), dtype=torch.float32, device=T.device)
        if grad_invdepth is None:
            grad_invdepth = torch.zeros_like(T)
        g = ctx.renderer.backward(ctx.frame, ctx.scene, ctx.cam, T, nc, grad_rgb, dL_dinvdepth=grad_invdepth)
        ctx.renderer.release_frame(ctx.frame)
        ctx.frame = None
        return (None, None, g["means"], g["log_scales"], g["quats"], g["opacity_logits"], g["sh"])


_default = {}


def render(scene: GaussianScene, cam, device: int = 0, blend_variant: int = 0):
    """Forward render with a per-device default renderer; returns (rgb, T, n_contrib)."""
    r = _default.get(device)
    if r is None:
        r = _default[device] = Renderer(device)
    frame = r.acquire_frame()
    rgb, T, nc, _ = r.forward(scene, cam, frame=frame, blend_variant=blend_variant)
    r.release_frame(frame)
    return rgb, T, nc
