"""The C-ABI library loads, exports every declared entry point, and rejects
bad arguments before touching a device (no GPU needed)."""
import ctypes
import os
import re

import pytest

from paper_2509_25626_amd import native

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cdnasplat.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(cds_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(native.LIB_PATH):
        from paper_2509_25626_amd import build
        build.build()
    return native.load()


def test_every_declared_symbol_is_exported(lib):
    names = _declared()
    assert len(names) >= 20
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    # and the binding describes each one
    assert set(names) == set(native.SIGNATURES), set(names) ^ set(native.SIGNATURES)


def test_version_and_error_text(lib):
    assert b"cdnasplat" in lib.cds_version()
    assert lib.cds_last_error() is not None


def test_null_arguments_rejected_without_device_work(lib):
    P = ctypes.c_void_p
    assert lib.cds_create(None, 0, None) == native.CDS_ERR_INVALID_ARG
    assert lib.cds_render_forward(None, None, None, None, None, None, None, None, None) == \
        native.CDS_ERR_INVALID_ARG
    assert b"NULL" in lib.cds_last_error()
    assert lib.cds_render_backward(None, None, None, None, None, None, None, None, None) == \
        native.CDS_ERR_INVALID_ARG
    assert lib.cds_sort_pairs(None, None, None, 10, 64, None, None, 0, None) == native.CDS_ERR_INVALID_ARG
    assert lib.cds_exclusive_scan_u32(None, None, 10, None, None, None) == native.CDS_ERR_INVALID_ARG
    assert lib.cds_frame_create(None, ctypes.byref(P())) == native.CDS_ERR_INVALID_ARG
    assert lib.cds_frame_get_info(None, None) == native.CDS_ERR_INVALID_ARG
    assert lib.cds_check_device(None, None) == native.CDS_ERR_INVALID_ARG
    assert lib.cds_l1_loss_grad(None, None, None, 4, None, None, None) == native.CDS_ERR_INVALID_ARG
    lib.cds_destroy(None)
    lib.cds_frame_release(None)


def test_create_reports_missing_device_as_status(lib):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    h = ctypes.c_void_p()
    st = lib.cds_create(ctypes.byref(h), 0, None)
    assert st in (native.CDS_ERR_DEVICE, native.CDS_ERR_INVALID_ARG)
    assert not h.value


def test_header_constants_match_the_binding():
    """Every #define CDS_* integer in the header has the same value in the
    Python binding (option flags, status codes, limits)."""
    text = open(HEADER).read()
    defs = dict((k, int(v.rstrip("uU"), 0)) for k, v in
                re.findall(r"#define\s+(CDS_[A-Z0-9_]+)\s+(0x[0-9a-fA-F]+|\d+)u?\b", text))
    assert "CDS_OPT_KEEP_FOR_BACKWARD" in defs
    mismatched = {k: (v, getattr(native, k)) for k, v in defs.items()
                  if hasattr(native, k) and getattr(native, k) != v}
    assert not mismatched, mismatched
    for k in ("CDS_OPT_STAGE_TIMING", "CDS_OPT_SORT_ONESWEEP", "CDS_OPT_SORT_REDUCE_SCAN",
              "CDS_OPT_KEEP_FOR_BACKWARD"):
        assert hasattr(native, k), k
