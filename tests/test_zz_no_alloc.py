"""The allocation-free sort entry point (cds_sort_pairs_noalloc) against the
allocating one (cds_sort_pairs), through the C ABI: bit-identical keys and
values on two calls in a row, the second smaller, with no allocation made
through the context's allocator; sizes past its fixed maximum are refused."""
import ctypes

import numpy as np
import pytest
import torch

from paper_2509_25626_amd import native
from tests.conftest import gpu_available

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]


class CountingAllocator:
    """Device allocator backed by torch tensors that counts what it grants."""

    def __init__(self):
        self.granted = 0
        self.live = {}
        self._a = native.CdsAllocator._fields_[0][1](self._alloc)
        self._f = native.CdsAllocator._fields_[1][1](self._free)
        self.struct = native.CdsAllocator(self._a, self._f, None)

    def _alloc(self, nbytes, _user):
        t = torch.empty(int(nbytes), dtype=torch.uint8, device="cuda")
        self.granted += 1
        self.live[t.data_ptr()] = t
        return t.data_ptr()

    def _free(self, ptr, _user):
        self.live.pop(ptr, None)


def _pairs(count, end_bit, seed):
    rng = np.random.default_rng(seed)
    keys = rng.integers(0, 2**63, size=count, dtype=np.uint64) & np.uint64(0xFFFF0000000F00FF)
    keys[rng.random(count) < 0.3] = np.uint64(7)  # ties: stability matters
    vals = rng.permutation(count).astype(np.uint32)
    return keys, vals


def _sort(L, fn, ctx, keys, vals, end_bit, flags):
    kin = torch.from_numpy(keys.view(np.int64)).cuda()
    vin = torch.from_numpy(vals.view(np.int32)).cuda()
    kout = torch.full_like(kin, -1)
    vout = torch.full_like(vin, -1)
    stream = torch.cuda.current_stream().cuda_stream
    st = getattr(L, fn)(ctx, kin.data_ptr(), vin.data_ptr(), keys.size, end_bit, kout.data_ptr(),
                        vout.data_ptr(), flags, stream)
    native.check(st)
    native.check(L.cds_check_device(ctx, stream))
    # inputs untouched
    assert np.array_equal(kin.cpu().numpy().view(np.uint64), keys)
    return kout.cpu().numpy().view(np.uint64), vout.cpu().numpy().view(np.uint32)


@pytest.mark.parametrize("flags", [0, native.CDS_OPT_SORT_REDUCE_SCAN])
def test_noalloc_sort_matches_allocating_sort(flags):
    L = native.load()
    alloc = CountingAllocator()
    ctx = ctypes.c_void_p()
    native.check(L.cds_create(ctypes.byref(ctx), 0, ctypes.byref(alloc.struct)))
    try:
        # a large call, then a smaller one: the second reuses what the first left behind
        for count, end_bit, seed in ((native.CDS_NOALLOC_MAX_PAIRS, 64, 1), (123_457, 44, 2), (4097, 12, 3)):
            keys, vals = _pairs(count, end_bit, seed)
            ref_k, ref_v = _sort(L, "cds_sort_pairs", ctx, keys, vals, end_bit, flags)
            before = alloc.granted
            got_k, got_v = _sort(L, "cds_sort_pairs_noalloc", ctx, keys, vals, end_bit, flags)
            assert alloc.granted == before, "the allocation-free sort allocated"
            assert np.array_equal(got_k, ref_k) and np.array_equal(got_v, ref_v), (count, end_bit)
            # and both equal a stable sort on the key bits
            mask = np.uint64((1 << end_bit) - 1) if end_bit < 64 else np.uint64(0xFFFFFFFFFFFFFFFF)
            order = np.argsort(keys & mask, kind="stable")
            assert np.array_equal(got_k, keys[order]) and np.array_equal(got_v, vals[order])
    finally:
        L.cds_destroy(ctx)
        torch.cuda.synchronize()


def test_noalloc_sort_limits():
    L = native.load()
    ctx = ctypes.c_void_p()
    native.check(L.cds_create(ctypes.byref(ctx), 0, None))
    try:
        big = native.CDS_NOALLOC_MAX_PAIRS + 1
        p = ctypes.c_void_p(16)  # never dereferenced: the size check comes first
        assert L.cds_sort_pairs_noalloc(ctx, p, p, big, 64, p, p, 0, None) == native.CDS_ERR_CAPACITY
        assert b"at most" in L.cds_last_error()
        assert L.cds_sort_pairs_noalloc(ctx, None, None, 0, 64, None, None, 0, None) == native.CDS_OK
        assert L.cds_sort_pairs_noalloc(None, None, None, 0, 64, None, None, 0, None) == \
            native.CDS_ERR_INVALID_ARG
    finally:
        L.cds_destroy(ctx)
