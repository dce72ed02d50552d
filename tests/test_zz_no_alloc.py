"""gsr_raster_batch_noalloc (the batched raster whose work-item list lives in the
library's device-resident scratch) against gsr_raster_batch (the same launch with a
caller workspace), called through the C ABI: bitwise equal images, on two calls in
a row, the second with a smaller batch; a batch above the scratch's tile limit is
rejected before any launch."""
import ctypes

import numpy as np
import pytest
import torch

from helpers import ensure_built
from paper_2503_01199_amd import scenes

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rz():
    ensure_built()
    from paper_2503_01199_amd.raster import Rasterizer
    return Rasterizer(0)


def _tables(frames, device):
    n = len(frames)
    wsp = (ctypes.c_void_p * n)(*[f.workspace.ptr for f in frames])
    images = [[torch.full((3, c.height, c.width), -1.0, dtype=torch.float32, device=device) for c in f.cameras]
              for f in frames]
    rows = [(ctypes.c_void_p * len(im))(*[t.data_ptr() for t in im]) for im in images]
    table = (ctypes.POINTER(ctypes.c_void_p) * n)(*[ctypes.cast(r, ctypes.POINTER(ctypes.c_void_p)) for r in rows])
    return wsp, images, rows, table


def _noalloc(rz, frames, precision):
    wsp, images, rows, table = _tables(frames, rz.device)
    st = rz.lib.gsr_raster_batch_noalloc(rz.ctx, len(frames), wsp, table, int(precision), rz._stream())
    rz._check(st, "gsr_raster_batch_noalloc")
    torch.cuda.synchronize()
    return [[t.cpu().numpy() for t in im] for im in images]


def _with_workspace(rz, frames, precision):
    from paper_2503_01199_amd.raster import Workspace
    wsp, images, rows, table = _tables(frames, rz.device)
    nbytes = ctypes.c_size_t()
    rz._check(rz.lib.gsr_raster_batch_workspace_size(rz.ctx, len(frames), wsp, ctypes.byref(nbytes)), "size")
    bws = Workspace(rz.device)
    bws.ensure(max(nbytes.value, 256))
    st = rz.lib.gsr_raster_batch(rz.ctx, len(frames), wsp, table, int(precision), bws.ptr, bws.nbytes, rz._stream())
    rz._check(st, "gsr_raster_batch")
    torch.cuda.synchronize()
    return [[t.cpu().numpy() for t in im] for im in images]


def _prepare(rz, specs):
    from paper_2503_01199_amd.raster import SceneTensors, Workspace
    frames = []
    for sc, cams in specs:
        st = SceneTensors.from_scene(sc, rz.device)
        frames.append(rz.prepare(st, cams, workspace=Workspace(rz.device)))
    torch.cuda.synchronize()
    for f in frames:
        rz.check_frame(f)
    return frames


@pytest.mark.parametrize("precision", [0, 1])
def test_noalloc_batch_equals_workspace_batch_twice(rz, precision):
    big = scenes.spheres_planes_scene(60_000, seed_salt=2)
    tiny = scenes.tiny_scene(6000, seed_salt=9)
    first = [(big, [scenes.orbit_camera(20.0, 10.0, radius=7.0, width=640, height=480),
                    scenes.orbit_camera(110.0, 5.0, radius=7.0, width=320, height=200)]),
             (tiny, [scenes.tiny_camera(128, 128)]),
             (tiny, [scenes.tiny_camera(100, 75)])]
    second = [(tiny, [scenes.tiny_camera(100, 75)])]  # a smaller batch on the same scratch
    for what, specs in (("first", first), ("second", second)):
        print("no-alloc batch, %s call, precision %d" % (what, precision), flush=True)
        frames = _prepare(rz, specs)
        a = _noalloc(rz, frames, precision)
        b = _with_workspace(rz, frames, precision)
        for fa, fb in zip(a, b):
            for ia, ib in zip(fa, fb):
                assert (ia != -1.0).all()  # every pixel written
                assert np.array_equal(ia.view(np.uint32), ib.view(np.uint32))


def test_noalloc_batch_rejects_more_tiles_than_its_scratch(rz):
    from paper_2503_01199_amd import _lib as L
    tiny = scenes.tiny_scene(64, seed_salt=1)
    # one view of 8208 x 8192 pixels: 513 x 512 = 262,656 tiles > 262,144
    frames = _prepare(rz, [(tiny, [scenes.tiny_camera(8208, 8192)])])
    wsp, images, rows, table = _tables(frames, rz.device)
    st = rz.lib.gsr_raster_batch_noalloc(rz.ctx, 1, wsp, table, 0, rz._stream())
    assert st == L.GSR_ERR_INVALID_ARG
    assert b"scratch" in rz.lib.gsr_last_error(rz.ctx)
