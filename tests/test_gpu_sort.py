"""The one-sweep radix sort (gsr_sort_u32) against numpy's stable argsort, bit for
bit: 2^24 + 3 random 32-bit keys (the path of 4096-item tiles and 16-byte histogram
loads that sorts of 16M or more items take), the same keys from an address 4 bytes
past a 16-byte boundary (the histogram's per-key fallback), 16-bit keys with heavy
ties (tile ids: stability decides the order), ragged small sizes (also either
side of a full look-back group) and argument errors."""
import numpy as np
import pytest
import torch

from helpers import ensure_built

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rz():
    ensure_built()
    from paper_2503_01199_amd.raster import Rasterizer
    return Rasterizer(0)


def _check(rz, keys_np, vals_np, bits, offset=0):
    n = len(keys_np)
    buf = torch.zeros(n + offset, dtype=torch.int32, device=rz.device)
    buf[offset:] = torch.as_tensor(keys_np.view(np.int32), device=rz.device)
    keys = buf[offset:]
    vals = None if vals_np is None else torch.as_tensor(vals_np.view(np.int32), device=rz.device)
    print("sort n=%d bits=%d offset=%d values=%s" % (n, bits, offset, vals_np is not None), flush=True)
    ok, ov = rz.sort_u32(keys, vals, bits)
    torch.cuda.synchronize()
    order = np.argsort(keys_np, kind="stable")
    want_v = order.astype(np.uint32) if vals_np is None else vals_np[order]
    got_k = ok.cpu().numpy().view(np.uint32)
    got_v = ov.cpu().numpy().view(np.uint32)
    assert np.array_equal(got_k, keys_np[order])
    assert np.array_equal(got_v, want_v)


def test_sort_large_random_keys(rz):
    rng = np.random.default_rng(11)
    n = (1 << 24) + 3
    keys = rng.integers(0, 1 << 32, size=n, dtype=np.uint64).astype(np.uint32)
    vals = rng.integers(0, 1 << 32, size=n, dtype=np.uint64).astype(np.uint32)
    _check(rz, keys, vals, 32)
    _check(rz, keys, vals, 32, offset=1)  # keys 4 bytes past a 16-byte boundary


def test_sort_large_tile_ids_stable(rz):
    rng = np.random.default_rng(12)
    n = (1 << 24) + 1000
    keys = rng.integers(0, 65280, size=n).astype(np.uint32)
    _check(rz, keys, None, 16)


# 2048-item tiles below 2^24 items, in look-back groups of 32 tiles: 65,536 items
# fill exactly one group, one more item opens a second group with one tile
@pytest.mark.parametrize("n,bits", [(1, 32), (7, 8), (2049, 13), (4097, 24), (65_535, 32), (65_536, 32),
                                    (65_537, 16), (131_073, 32), (300_001, 32)])
def test_sort_small_and_ragged(rz, n, bits):
    rng = np.random.default_rng(13 + n)
    keys = rng.integers(0, 1 << bits, size=n, dtype=np.uint64).astype(np.uint32)
    keys[: n // 3] = keys[0]  # ties
    vals = np.arange(n, dtype=np.uint32)[::-1].copy()
    _check(rz, keys, vals, bits)


def test_sort_argument_errors(rz):
    from paper_2503_01199_amd import _lib as L
    k = torch.zeros(16, dtype=torch.int32, device=rz.device)
    for bits in (0, 33):
        with pytest.raises(L.GsrError) as e:
            rz.sort_u32(k, None, bits)
        assert e.value.status == L.GSR_ERR_INVALID_ARG
    out = torch.zeros(16, dtype=torch.int32, device=rz.device)
    import ctypes
    nb = ctypes.c_size_t()
    assert rz.lib.gsr_sort_workspace_size(rz.ctx, 16, 32, ctypes.byref(nb)) == 0
    from paper_2503_01199_amd.raster import Workspace
    ws = Workspace(rz.device)
    ws.ensure(nb.value)
    # outputs overlapping the input are rejected before any launch
    st = rz.lib.gsr_sort_u32(rz.ctx, k.data_ptr(), None, 16, 32, k.data_ptr(), out.data_ptr(), ws.ptr, ws.nbytes,
                             None)
    assert st == L.GSR_ERR_INVALID_ARG
    st = rz.lib.gsr_sort_u32(rz.ctx, k.data_ptr(), None, 16, 32, out.data_ptr(), out.data_ptr() + 8, ws.ptr,
                             ws.nbytes, None)
    assert st == L.GSR_ERR_INVALID_ARG
    out2 = torch.zeros(16, dtype=torch.int32, device=rz.device)
    st = rz.lib.gsr_sort_u32(rz.ctx, k.data_ptr(), None, 16, 32, out.data_ptr(), out2.data_ptr(), ws.ptr, 64, None)
    assert st == L.GSR_ERR_WORKSPACE_TOO_SMALL
