"""The 3-sigma tile-membership bound (gsr_options.radius_mode = 1) against the
oracle under the same bound: rects and sorted instances bit-exact (except rects
the oracle flags as within rounding of a pixel-centre boundary), images within
1e-5 on non-fragile pixels, every gradient and S, M per element within 1e-3 and C
within the oracle's slack. Under this bound a pixel blends a Gaussian only if its
tile is in the Gaussian's rect, so images differ from the default bound's."""
import numpy as np
import pytest
import torch

import oracle as orc
from helpers import GRAD_TOL, IMAGE_TOL, ensure_built, grad_errors, image_errors
from paper_2503_01199_amd import scenes
from parity import GROUPS, compare_counts

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rz():
    ensure_built()
    from paper_2503_01199_amd.raster import Rasterizer
    return Rasterizer(0)


def _case(which):
    if which == "tiny":
        return scenes.tiny_scene(), scenes.tiny_camera()
    if which == "ragged":
        return scenes.tiny_scene(3000, seed_salt=4), scenes.tiny_camera(100, 75)
    sc = scenes.spheres_planes_scene(40_000, seed_salt=6)
    _, perm = orc.morton(sc.means)
    sc = sc.permuted(perm)
    cam = scenes.spheres_planes_camera()
    cam.width, cam.height, cam.cx, cam.cy = 400, 300, 200.0, 150.0
    cam.fx = cam.fy = float(np.float32(cam.fx * 0.5))
    return sc, cam


@pytest.mark.parametrize("which", ["tiny", "ragged", "spheres"])
def test_three_sigma_bound_matches_oracle(rz, which):
    from paper_2503_01199_amd.raster import SceneTensors, Workspace, new_stats
    sc, cam = _case(which)
    ref = orc.render(sc, cam, mode=1, radius_mode=1)
    w, gt = scenes.l1_weights((3, cam.height, cam.width), config=0, salt=17)
    g = orc.l1_grad(ref["image"], w, gt).astype(np.float32)
    g[:, ref["fragile"]] = 0.0
    print("radius_mode 1 %s n=%d" % (which, sc.n), flush=True)
    st = SceneTensors.from_scene(sc, rz.device)
    fr = rz.forward(st, [cam], workspace=Workspace(rz.device), radius_mode=1)
    stats = new_stats(sc.n, rz.device)
    grads = rz.backward(fr, [torch.as_tensor(g, device=rz.device)], stats=stats)
    torch.cuda.synchronize()
    # rects against the oracle's 3-sigma rects
    ins = rz.inspect(fr)
    pp = orc.preprocess(sc, cam, radius_mode=1)
    c2f = ins["compact2full"].cpu().numpy().view(np.uint32).astype(np.int64)
    live = c2f != 0xFFFFFFFF
    rect = ins["rect"].cpu().numpy().view(np.uint16).astype(np.int64)[live]
    ntile = ins["tiles"].cpu().numpy().view(np.uint32)[live]
    full = c2f[live]
    valid = pp["valid"][full]
    ok = ~pp["rect_fragile"][full]
    assert np.array_equal(ntile > 0, valid)
    chk = valid & ok
    assert np.array_equal(rect[chk], pp["rect"][full][chk])
    print("rects equal on %d Gaussians (%d within rounding skipped)" % (chk.sum(), (valid & ~ok).sum()))
    # the default bound gives another instance count (the bounds differ on this scene)
    fr0 = rz.forward(st, [cam], workspace=Workspace(rz.device))
    print("instances: 3-sigma %d, opacity-aware %d" % (fr.info["instances"], fr0.info["instances"]))
    assert fr.info["instances"] != fr0.info["instances"]
    # image and per-pixel state
    err, over, nfrag = image_errors(fr.images[0].cpu().numpy(), ref["image"], ref["fragile"])
    print("radius_mode 1 %s: image max rel %.3g (%d fragile pixels)" % (which, err, nfrag))
    assert err <= IMAGE_TOL
    # gradients, statistic
    ob = orc.backward(sc, cam, g.astype(np.float64), mode=1, radius_mode=1)
    none = np.zeros(sc.n, bool)
    for k in GROUPS:
        e = grad_errors(grads[k].cpu().numpy(), ob[k], none)
        print("  %-15s max rel %.3g" % (k, e))
        assert e <= GRAD_TOL, k
    S = {k: v.cpu().numpy() for k, v in stats.items()}
    for k in ("M", "S"):
        assert grad_errors(S[k], ob[k], none) <= GRAD_TOL, k
    compare_counts(S["C"], ob, "radius_mode 1 %s" % which)


def test_radius_mode_is_validated(rz):
    from paper_2503_01199_amd import _lib as L
    from paper_2503_01199_amd.raster import SceneTensors, Workspace
    sc, cam = scenes.tiny_scene(), scenes.tiny_camera()
    with pytest.raises(L.GsrError) as e:
        rz.forward(SceneTensors.from_scene(sc, rz.device), [cam], workspace=Workspace(rz.device), radius_mode=2)
    assert e.value.status == L.GSR_ERR_INVALID_ARG
