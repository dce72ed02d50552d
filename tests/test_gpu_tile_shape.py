"""Tiles of 256 pixels in other shapes than 16x16 (gsr_options.tile_width; Sec. 3.1
treats the tile shape and the pixels per thread as parameters of the raster) against
the FP64 oracle: instance keys, values and tile ranges bit for bit against the oracle
binned on the same tile grid, images and gradients at the bars of the 16x16 path
(the image and the gradients do not depend on the tile shape)."""
import numpy as np
import pytest
import torch

import oracle as orc
from helpers import ensure_built
from paper_2503_01199_amd import scenes
from parity import compare, compare_images, oracle_sum, upstream

pytestmark = pytest.mark.gpu

SHAPES = [4, 8, 32, 64]


@pytest.fixture(scope="module")
def rz():
    ensure_built()
    from paper_2503_01199_amd.raster import Rasterizer
    return Rasterizer(0)


def _forward(rz, sc, cams, tw, deterministic=False):
    from paper_2503_01199_amd.raster import SceneTensors, Workspace
    print("tile width %d: forward n=%d views=%s" % (tw, sc.n, [(c.width, c.height) for c in cams]), flush=True)
    st = SceneTensors.from_scene(sc, rz.device)
    fr = rz.forward(st, cams, workspace=Workspace(rz.device), tile_width=tw, deterministic=deterministic)
    torch.cuda.synchronize()
    return fr


def _fwd_bwd(rz, sc, cams, gI, tw, deterministic=False):
    from paper_2503_01199_amd.raster import new_stats
    fr = _forward(rz, sc, cams, tw, deterministic)
    stats = new_stats(sc.n, rz.device)
    grads = rz.backward(fr, [torch.as_tensor(g, device=rz.device) for g in gI], stats=stats)
    torch.cuda.synchronize()
    return fr, {k: v.cpu().numpy() for k, v in grads.items()}, {k: v.cpu().numpy() for k, v in stats.items()}


def _oracle_bins(sc, cams, tw):
    th = 256 // tw
    views = []
    for cam in cams:
        pp = orc.preprocess(sc, cam, tile_width=tw)
        assert not pp["rect_fragile"].any()
        views.append((pp["valid"], pp["rect"], pp["depth_bits"], -(-cam.width // tw), -(-cam.height // th)))
    return orc.bin_instances(views)


@pytest.mark.parametrize("tw", SHAPES)
def test_binning_bit_exact(rz, tw):
    """Two views with ragged edges in both axes for every shape."""
    sc = scenes.tiny_scene(800, seed_salt=4)
    cams = [scenes.tiny_camera(100, 75), scenes.tiny_camera(72, 40)]
    fr = _forward(rz, sc, cams, tw)
    ins = rz.inspect(fr)
    keys, vals, ranges = _oracle_bins(sc, cams, tw)
    V = len(cams)
    assert ins["info"]["instances"] == len(keys)
    assert ins["info"]["tiles"] == np.asarray(ranges).reshape(-1, 2).shape[0]
    c2f = ins["compact2full"].cpu().numpy().view(np.uint32).astype(np.int64)
    R = ins["records"].shape[0]
    slots, view = np.arange(R) // V, np.arange(R) % V
    full = np.where(c2f[slots] == 0xFFFFFFFF, -1, c2f[slots])
    it = ins["inst_tile"].cpu().numpy().view(np.uint32).astype(np.uint64)
    ir = ins["inst_record"].cpu().numpy().view(np.uint32).astype(np.int64)
    dk = ins["depth_key"].cpu().numpy().view(np.uint32).astype(np.uint64)
    assert np.array_equal((it << np.uint64(32)) | dk[ir], keys)
    assert np.array_equal(view[ir] * sc.n + full[ir], vals)
    assert np.array_equal(ins["ranges"].cpu().numpy().view(np.uint32), ranges)


@pytest.mark.parametrize("tw", SHAPES)
def test_images_and_gradients(rz, tw):
    sc, cam = scenes.tiny_scene(), scenes.tiny_camera(100, 90)
    gI, refs = upstream(sc, [cam])
    fr, grads, stats = _fwd_bwd(rz, sc, [cam], gI, tw)
    what = "tiles %dx%d" % (tw, 256 // tw)
    compare_images(fr, refs, what)
    compare(grads, stats, oracle_sum(sc, [cam], gI), what, logits=sc.opacity_logits)


@pytest.mark.parametrize("tw", SHAPES)
def test_split_tiles(rz, tw):
    """6,000 Gaussians on a small image: the longest lists run as band items (one
    pixel per lane in the forward, two in the backward) of every shape."""
    sc = scenes.tiny_scene(6000, seed_salt=9)
    cam = scenes.tiny_camera(100, 75)
    gI, refs = upstream(sc, [cam])
    fr, grads, stats = _fwd_bwd(rz, sc, [cam], gI, tw)
    info = rz.inspect(fr)["info"]
    print("split tiles: forward %d, backward %d" % (info["split_tiles"], info["split_tiles_bwd"]))
    assert info["split_tiles"] > 0 and info["split_tiles_bwd"] > 0
    what = "split tiles %dx%d" % (tw, 256 // tw)
    compare_images(fr, refs, what)
    compare(grads, stats, oracle_sum(sc, [cam], gI), what, logits=sc.opacity_logits)


def test_width_16_is_the_default(rz):
    """tile_width 16 and 0 are the same frame: image and gradients bit for bit (the
    gradients summed in fixed point, so that the order of the tiles' atomics does
    not enter)."""
    sc, cam = scenes.tiny_scene(), scenes.tiny_camera(100, 90)
    gI, _ = upstream(sc, [cam])
    out = [_fwd_bwd(rz, sc, [cam], gI, tw, deterministic=True) for tw in (0, 16)]
    assert torch.equal(out[0][0].images[0], out[1][0].images[0])
    for k in out[0][1]:
        assert np.array_equal(out[0][1][k], out[1][1][k]), k


def test_bad_tile_width_and_mismatched_backward_rejected(rz):
    from paper_2503_01199_amd import _lib as L
    sc, cam = scenes.tiny_scene(), scenes.tiny_camera()
    with pytest.raises(L.GsrError):
        _forward(rz, sc, [cam], 12)
    fr = _forward(rz, sc, [cam], 8)
    fr.opts.tile_width = 32
    g = torch.zeros((3, cam.height, cam.width), dtype=torch.float32, device=rz.device)
    with pytest.raises(L.GsrError, match="tile_width"):
        rz.backward(fr, [g])
