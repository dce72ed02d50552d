"""The error path of the device-wide waits, forced from the host.

Every scan and sort wait is bounded by elapsed time (100 ms) and reads the frame's
error word on each round; the first wait that runs out raises the abort bit, and
every other wait and every later kernel of the frame leaves when it is set. These
tests force the condition from the host, so that every kernel still exits
normally: (1) the abort bit raised before the depth sort; (2) a block of the tile
sort's first pass that never publishes its look-back status, so that the waits
behind it can only end by their time bound. In both cases gsr_frame_inspect must
return GSR_ERR_DEVICE within a fraction of a second, a backward on the aborted
frame must run without touching memory it should not, and the next frame on the
same workspace must render exactly as before.
"""
import time

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


@pytest.mark.parametrize("mode", ["abort_before_sort", "withhold_status"])
def test_aborted_frame_surfaces_promptly(rz, mode):
    from paper_2503_01199_amd import _lib as L
    from paper_2503_01199_amd.raster import SceneTensors, Workspace
    sc = scenes.tiny_scene(6000, seed_salt=9)
    cam = scenes.tiny_camera()
    st = SceneTensors.from_scene(sc, rz.device)
    ws = Workspace(rz.device)
    print("abort test %s: good frame" % mode, flush=True)
    good = rz.forward(st, [cam], workspace=ws)
    torch.cuda.synchronize()
    img0 = good.images[0].clone()
    # the tile sort's first pass has more than three 2048-instance tiles, so tile 1 has
    # successors that wait on it
    assert good.info["instances"] > 3 * 2048, good.info
    code = {"abort_before_sort": L.GSR_FAULT_ABORT_BEFORE_SORT,
            "withhold_status": L.GSR_FAULT_WITHHOLD_STATUS}[mode]
    rz.set_fault_injection(code)
    try:
        print("abort test %s: injected frame" % mode, flush=True)
        t0 = time.perf_counter()
        fr = rz.forward(st, [cam], workspace=ws, check=False)
        with pytest.raises(L.GsrError) as e:
            rz.check_frame(fr)
        dt = time.perf_counter() - t0
        print("abort test %s: %s after %.3f s" % (mode, e.value, dt), flush=True)
        assert e.value.status == L.GSR_ERR_DEVICE
        assert dt < 2.0
        # a backward on the aborted frame: every kernel leaves at once
        zero = torch.zeros((3, cam.height, cam.width), device=rz.device)
        rz.backward(fr, [zero])
        torch.cuda.synchronize()
    finally:
        rz.set_fault_injection(L.GSR_FAULT_NONE)
    print("abort test %s: next frame" % mode, flush=True)
    again = rz.forward(st, [cam], workspace=ws)
    torch.cuda.synchronize()
    assert torch.equal(again.images[0], img0)
    assert again.info == good.info


def test_fault_injection_rejects_unknown_modes(rz):
    from paper_2503_01199_amd import _lib as L
    with pytest.raises(L.GsrError) as e:
        rz.set_fault_injection(7)
    assert e.value.status == L.GSR_ERR_INVALID_ARG
    rz.set_fault_injection(L.GSR_FAULT_NONE)
