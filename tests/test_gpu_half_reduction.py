"""The half2-packed colour/opacity gradient reduction (gsr_options.half_reduction,
Sec. 3.1.2): an approximation whose error against the FP64 oracle is reported.

Each lane's colour and opacity sums are rounded to FP16 (relative 2^-11), reduced
over the wave in packed FP16 (six adds, each rounding relative to its partial
sum) and added across tiles with packed FP16 atomics (a record touches a few tiles
here). A colour or opacity gradient is then off by a few 2^-11 of the magnitudes
summed, so the sanity bounds below are normwise 1e-2 per group (the mean gradient
takes the colour's view-direction term, so it carries that error too) and 5e-2 on
the worst element relative to the group's largest. A per-element relative bound
would not hold: a Gaussian whose per-tile sums cancel keeps the FP16 rounding of
the terms, which can exceed its small final value. The screen-mean and conic
gradients and the square sum stay FP32, so S matches the FP32 path at the 1e-3
parity bar. Values below FP16's normal range (6.1e-5) lose relative precision: a
mean-reduced loss (upstream of order 1/(3HW)) is reported as well."""
import numpy as np
import pytest
import torch

import oracle as orc
from helpers import GRAD_TOL, ensure_built, grad_errors, normwise
from paper_2503_01199_amd import scenes
from parity import GROUPS, upstream

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rz():
    ensure_built()
    from paper_2503_01199_amd.raster import Rasterizer
    return Rasterizer(0)


def _run(rz, sc, cam, g, half):
    from paper_2503_01199_amd.raster import SceneTensors, Workspace, new_stats
    st = SceneTensors.from_scene(sc, rz.device)
    fr = rz.forward(st, [cam], workspace=Workspace(rz.device))
    fr.opts.half_reduction = 1 if half else 0
    stats = new_stats(sc.n, rz.device)
    grads = rz.backward(fr, [torch.as_tensor(g, device=rz.device)], stats=stats)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in grads.items()}, {k: v.cpu().numpy() for k, v in stats.items()}


@pytest.mark.parametrize("which", ["tiny", "split", "spheres"])
def test_half_reduction_error_report(rz, which):
    if which == "tiny":
        sc, cam = scenes.tiny_scene(), scenes.tiny_camera()
    elif which == "split":
        sc, cam = scenes.tiny_scene(6000, seed_salt=9), scenes.tiny_camera()
    else:
        sc = scenes.spheres_planes_scene(30_000, seed_salt=3)
        _, perm = orc.morton(sc.means)
        sc = sc.permuted(perm)
        cam = scenes.spheres_planes_camera()
        cam.width, cam.height, cam.cx, cam.cy = 320, 240, 160.0, 120.0
        cam.fx = cam.fy = float(np.float32(cam.fx * 0.4))
    gI, _ = upstream(sc, [cam], salt=21)
    g = gI[0]
    print("half reduction %s n=%d" % (which, sc.n), flush=True)
    gh, sh = _run(rz, sc, cam, g, True)
    gf, sf = _run(rz, sc, cam, g, False)
    ob = orc.backward(sc, cam, g.astype(np.float64), mode=1)
    none = np.zeros(sc.n, bool)
    errs = {}
    for k in GROUPS:
        nw = normwise(gh[k], ob[k])
        mx = float(np.abs(gh[k] - ob[k]).max() / max(np.abs(ob[k]).max(), 1e-30))
        errs[k] = (nw, mx)
        print("  %s %-15s half: normwise %.3g worst/largest %.3g max rel %.3g | fp32: normwise %.3g"
              % (which, k, nw, mx, grad_errors(gh[k], ob[k], none), normwise(gf[k], ob[k])))
    for k, (nw, mx) in errs.items():
        assert nw < 1e-2 and mx < 5e-2, k
    print("  %s statistic M half: normwise %.3g; S max rel %.3g; C equal %s"
          % (which, normwise(sh["M"], ob["M"]), grad_errors(sh["S"], ob["S"], none),
             np.array_equal(sh["C"], sf["C"])))
    assert normwise(sh["M"], ob["M"]) < 1e-2
    assert grad_errors(sh["S"], ob["S"], none) <= GRAD_TOL
    assert np.array_equal(sh["C"], sf["C"])  # the count is exact in both layouts


def test_half_reduction_small_loss_scale_is_reported(rz):
    """A mean-reduced loss on the tiny scene: colour sums near FP16's subnormal
    range. Reported only."""
    sc, cam = scenes.tiny_scene(), scenes.tiny_camera()
    gI, _ = upstream(sc, [cam], salt=22)
    g = (gI[0] / np.float32(3 * cam.width * cam.height)).astype(np.float32)
    gh, _ = _run(rz, sc, cam, g, True)
    ob = orc.backward(sc, cam, g.astype(np.float64), mode=1)
    print("half reduction at a mean-reduced loss: " + ", ".join(
        "%s %.3g" % (k, normwise(gh[k], ob[k])) for k in GROUPS))


def test_half_reduction_excludes_deterministic(rz):
    from paper_2503_01199_amd import _lib as L
    from paper_2503_01199_amd.raster import SceneTensors, Workspace
    sc, cam = scenes.tiny_scene(), scenes.tiny_camera()
    fr = rz.forward(SceneTensors.from_scene(sc, rz.device), [cam], workspace=Workspace(rz.device),
                    deterministic=True)
    fr.opts.half_reduction = 1
    with pytest.raises(L.GsrError) as e:
        rz.backward(fr, [torch.zeros((3, cam.height, cam.width), device=rz.device)])
    assert e.value.status == L.GSR_ERR_INVALID_ARG
