"""ctypes binding of ``libcdnasplat.so`` (the C ABI in ``include/cdnasplat.h``).

Argument marshalling only: every step of the rendering pipeline runs in the
library's HIP kernels.  Loading fails loudly when the library has not been
built (``python -m paper_2509_25626_amd.build``); there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
import threading

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libcdnasplat.so")

CDS_OK, CDS_ERR_INVALID_ARG, CDS_ERR_OOM, CDS_ERR_CAPACITY, CDS_ERR_DEVICE, CDS_ERR_BUSY = range(6)
STATUS_NAMES = {0: "CDS_OK", 1: "CDS_ERR_INVALID_ARG", 2: "CDS_ERR_OOM", 3: "CDS_ERR_CAPACITY",
                4: "CDS_ERR_DEVICE", 5: "CDS_ERR_BUSY"}

P = ctypes.c_void_p


class CdsError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


class CdsAllocator(ctypes.Structure):
    _fields_ = [("alloc", ctypes.CFUNCTYPE(P, ctypes.c_size_t, P)),
                ("free", ctypes.CFUNCTYPE(None, P, P)),
                ("user", P)]


class CdsScene(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("sh_degree", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("means", P), ("log_scales", P), ("quats", P), ("opacity_logits", P), ("sh", P)]


class CdsSceneGrad(ctypes.Structure):
    _fields_ = [("means", P), ("log_scales", P), ("quats", P), ("opacity_logits", P), ("sh", P)]


class CdsCamera(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int32), ("height", ctypes.c_int32),
                ("fx", ctypes.c_float), ("fy", ctypes.c_float),
                ("cx", ctypes.c_float), ("cy", ctypes.c_float),
                ("view", ctypes.c_float * 12), ("near_plane", ctypes.c_float),
                ("bg", ctypes.c_float * 3)]


class CdsRenderOpts(ctypes.Structure):
    _fields_ = [("flags", ctypes.c_uint32), ("blend_variant", ctypes.c_int32),
                ("sort_variant", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class CdsFrameInfo(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("num_keys", ctypes.c_int64),
                ("width", ctypes.c_int32), ("height", ctypes.c_int32),
                ("tiles_x", ctypes.c_int32), ("tiles_y", ctypes.c_int32),
                ("sort_passes", ctypes.c_int32), ("num_visible", ctypes.c_int32),
                ("mean2d", P), ("conic_opacity", P), ("rgb", P), ("depth_bits", P),
                ("radius", P), ("tile_rect", P), ("tiles_touched", P), ("offsets", P),
                ("keys", P), ("values", P), ("ranges", P), ("clamp_flags", P),
                ("num_row_entries", ctypes.c_int64)]


class CdsStageTimes(ctypes.Structure):
    _fields_ = [(k, ctypes.c_float) for k in
                ("preprocess_ms", "scan_ms", "depth_order_ms", "duplicate_ms", "sort_ms", "ranges_ms",
                 "blend_ms", "blend_backward_ms", "preprocess_backward_ms", "sort_first_pass_ms")]


CDS_OPT_STAGE_TIMING = 1
CDS_OPT_SORT_ONESWEEP = 2
CDS_OPT_SORT_REDUCE_SCAN = 4
CDS_OPT_KEEP_FOR_BACKWARD = 8
CDS_NOALLOC_MAX_PAIRS = 1048576


class CdsServerOpts(ctypes.Structure):
    _fields_ = [("max_slots", ctypes.c_int32), ("max_batch", ctypes.c_int32),
                ("hbm_budget_bytes", ctypes.c_int64), ("sort_variant", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class CdsServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("completed", ctypes.c_int64),
                ("rejected", ctypes.c_int64), ("batches", ctypes.c_int64),
                ("workspace_bytes", ctypes.c_int64), ("peak_workspace_bytes", ctypes.c_int64),
                ("held_bytes", ctypes.c_int64), ("peak_held_bytes", ctypes.c_int64)]


# name -> (restype, argtypes)
SIGNATURES = {
    "cds_version": (ctypes.c_char_p, []),
    "cds_last_error": (ctypes.c_char_p, []),
    "cds_create": (ctypes.c_int, [ctypes.POINTER(P), ctypes.c_int, ctypes.POINTER(CdsAllocator)]),
    "cds_destroy": (None, [P]),
    "cds_frame_create": (ctypes.c_int, [P, ctypes.POINTER(P)]),
    "cds_frame_release": (None, [P]),
    "cds_render_forward": (ctypes.c_int, [P, P, ctypes.POINTER(CdsScene), ctypes.POINTER(CdsCamera),
                                          ctypes.POINTER(CdsRenderOpts), P, P, P, P]),
    "cds_render_backward": (ctypes.c_int, [P, P, ctypes.POINTER(CdsScene), ctypes.POINTER(CdsCamera),
                                           P, P, P, ctypes.POINTER(CdsSceneGrad), P]),
    "cds_render_forward_ex": (ctypes.c_int, [P, P, ctypes.POINTER(CdsScene), ctypes.POINTER(CdsCamera),
                                             ctypes.POINTER(CdsRenderOpts), P, P, P, P, P]),
    "cds_render_backward_ex": (ctypes.c_int, [P, P, ctypes.POINTER(CdsScene), ctypes.POINTER(CdsCamera),
                                              P, P, P, P, ctypes.POINTER(CdsSceneGrad), P]),
    "cds_l1_loss_grad": (ctypes.c_int, [P, P, P, ctypes.c_int64, P, P, P]),
    "cds_frame_get_info": (ctypes.c_int, [P, ctypes.POINTER(CdsFrameInfo)]),
    "cds_frame_stage_times": (ctypes.c_int, [P, ctypes.POINTER(CdsStageTimes)]),
    "cds_sort_pairs": (ctypes.c_int, [P, P, P, ctypes.c_int64, ctypes.c_int32, P, P, ctypes.c_uint32, P]),
    "cds_sort_pairs_noalloc": (ctypes.c_int, [P, P, P, ctypes.c_int64, ctypes.c_int32, P, P, ctypes.c_uint32, P]),
    "cds_exclusive_scan_u32": (ctypes.c_int, [P, P, ctypes.c_int64, P, P, P]),
    "cds_check_device": (ctypes.c_int, [P, P]),
    "cds_server_create": (ctypes.c_int, [P, ctypes.POINTER(CdsServerOpts), ctypes.POINTER(P)]),
    "cds_server_add_scene": (ctypes.c_int, [P, ctypes.POINTER(CdsScene), ctypes.POINTER(ctypes.c_int32)]),
    "cds_server_submit": (ctypes.c_int, [P, ctypes.c_int32, ctypes.POINTER(CdsCamera), P,
                                         ctypes.POINTER(ctypes.c_uint64)]),
    "cds_server_poll": (ctypes.c_int, [P, ctypes.c_uint64, ctypes.POINTER(ctypes.c_int32),
                                       ctypes.POINTER(ctypes.c_double)]),
    "cds_server_drain": (ctypes.c_int, [P]),
    "cds_server_get_stats": (ctypes.c_int, [P, ctypes.POINTER(CdsServerStats)]),
    "cds_server_destroy": (None, [P]),
}

_lib = None
_lock = threading.Lock()


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load the native library, or raise: the package has no non-HIP path."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(path):
                raise RuntimeError(
                    f"{path} is missing: build it with `python -m paper_2509_25626_amd.build` "
                    "(the renderer has no fallback implementation)")
            L = ctypes.CDLL(path)
            for name, (res, args) in SIGNATURES.items():
                fn = getattr(L, name)
                fn.restype = res
                fn.argtypes = args
            _lib = L
    return _lib


def check(status: int):
    if status != CDS_OK:
        msg = load().cds_last_error()
        raise CdsError(status, msg.decode() if msg else "")


def camera_struct(cam) -> CdsCamera:
    """C camera record from a scenes.Camera (or any object/dict with its fields)."""
    g = (lambda k: cam[k]) if isinstance(cam, dict) else (lambda k: getattr(cam, k))
    c = CdsCamera()
    c.width, c.height = int(g("width")), int(g("height"))
    c.fx, c.fy, c.cx, c.cy = (float(g(k)) for k in ("fx", "fy", "cx", "cy"))
    view = [float(v) for row in g("view") for v in (row if hasattr(row, "__len__") else [row])]
    if len(view) != 12:
        raise ValueError("view must be a 3x4 matrix")
    for i, v in enumerate(view):
        c.view[i] = v
    c.near_plane = float(g("near_plane"))
    for i, v in enumerate(g("bg")):
        c.bg[i] = float(v)
    return c
