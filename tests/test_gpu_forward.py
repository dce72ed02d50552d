"""GPU forward path vs the FP64 oracle: records, binning, image, per-pixel state.

Integer stages (depth keys, tile rects, sorted instances, tile ranges, list
positions) must match bit for bit; images within 1e-5 relative (floor 1) on pixels
that the oracle does not flag as fragile (a discrete decision within rounding of
its threshold).
"""
import numpy as np
import pytest
import torch

import oracle as orc
from helpers import IMAGE_TOL, decode_records, ensure_built, image_errors
from paper_2503_01199_amd import scenes

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rz():
    ensure_built()
    from paper_2503_01199_amd.raster import Rasterizer
    return Rasterizer(0)


def gpu_forward(rz, scene, cams, cull=True):
    from paper_2503_01199_amd.raster import SceneTensors, Workspace
    st = SceneTensors.from_scene(scene)
    print("gpu_forward n=%d views=%s cull=%s" % (scene.n, [(c.width, c.height) for c in cams], cull), flush=True)
    fr = rz.forward(st, cams, cluster_cull=cull, workspace=Workspace(rz.device))
    torch.cuda.synchronize()
    return fr


def full_index_of_records(ins, V):
    c2f = ins["compact2full"].cpu().numpy().view(np.uint32).astype(np.int64)
    R = ins["records"].shape[0]
    slots = np.arange(R) // V
    views = np.arange(R) % V
    full = np.where(c2f[slots] == 0xFFFFFFFF, -1, c2f[slots])
    return full, views


def check_image(fr, scene, cam, v=0, what=""):
    ref = orc.render(scene, cam, mode=2)
    img = fr.images[v].cpu().numpy()
    mx, bad, nfrag = image_errors(img, ref["image"], ref["fragile"])
    print("%s image max rel err %.3g, fragile pixels %d" % (what, mx, nfrag))
    assert nfrag <= max(2, 2e-3 * cam.width * cam.height)
    assert bad == 0, "%d pixels exceed %.0e (max %.3g)" % (bad, IMAGE_TOL, mx)
    return ref


@pytest.mark.parametrize("cull", [True, False])
def test_tiny_scene_image(rz, cull):
    sc, cam = scenes.tiny_scene(), scenes.tiny_camera()
    fr = gpu_forward(rz, sc, [cam], cull)
    check_image(fr, sc, cam, what="tiny cull=%s" % cull)


def test_records_match_oracle_projection(rz):
    sc, cam = scenes.tiny_scene(), scenes.tiny_camera()
    fr = gpu_forward(rz, sc, [cam])
    ins = rz.inspect(fr)
    pp = orc.preprocess(sc, cam)
    full, _ = full_index_of_records(ins, 1)
    tiles = ins["tiles"].cpu().numpy().view(np.uint32)
    valid_gpu = np.zeros(sc.n, bool)
    has = full >= 0
    valid_gpu[full[has]] = tiles[has] > 0
    assert np.array_equal(valid_gpu, pp["valid"])
    sel = has & (tiles > 0)
    g = full[sel]
    # depth key: FP32 bits of t_z, bit-exact
    dk = ins["depth_key"].cpu().numpy().view(np.uint32)[sel]
    assert np.array_equal(dk, pp["depth_bits"][g])
    # tile rect: exact except where an edge is within 1e-9 px of a pixel-centre boundary
    rect = ins["rect"].cpu().numpy().view(np.uint16).astype(np.int32)[sel]
    ok = np.all(rect == pp["rect"][g], axis=1) | pp["rect_fragile"][g]
    assert ok.all()
    assert np.array_equal(tiles[sel], pp["tiles"][g])
    u, v, conic, o, rgb = decode_records(ins["records"].cpu().numpy()[sel])
    assert np.abs(u - pp["u"][g]).max() < 1e-9 * 128 and np.abs(v - pp["v"][g]).max() < 1e-9 * 128
    rel = np.abs(conic - pp["conic"][g]) / np.abs(pp["conic"][g]).max(1, keepdims=True)
    assert rel.max() < 4e-7
    assert np.abs(o - pp["opacity"][g]).max() < 1e-7
    assert np.abs(rgb - pp["rgb"][g]).max() < 2e-7


def _oracle_bins(scene, cams):
    views = []
    for cam in cams:
        pp = orc.preprocess(scene, cam)
        tx, ty = cam.tiles()
        views.append((pp["valid"], pp["rect"], pp["depth_bits"], tx, ty))
        assert not pp["rect_fragile"].any()
    return orc.bin_instances(views)


def _large_footprint_scene():
    """The 800-Gaussian tiny scene with every 7th Gaussian 7.4x larger (log-scale + 2):
    footprints of tens of tiles up to whole small views."""
    sc = scenes.tiny_scene(800, seed_salt=4)
    big = np.arange(sc.n) % 7 == 0
    sc.log_scales[big] = sc.log_scales[big] + np.float32(2.0)
    return sc


@pytest.mark.parametrize("sizes", [[(320, 240)], [(128, 128), (200, 120)]])
def test_binning_bit_exact_large_footprints(rz, sizes):
    """Records of more than 4 tiles are emitted by whole waves (lanes on consecutive
    positions), several per wave here; the instance lists stay bit-exact."""
    sc = _large_footprint_scene()
    cams = [scenes.tiny_camera(w, h) for w, h in sizes]
    fr = gpu_forward(rz, sc, cams)
    ins = rz.inspect(fr)
    tiles = ins["tiles"].cpu().numpy().view(np.uint32)
    print("records with more than 16 tiles: %d (largest %d)" % ((tiles > 16).sum(), tiles.max()))
    assert (tiles > 16).sum() > 20
    keys, vals, ranges = _oracle_bins(sc, cams)
    assert ins["info"]["instances"] == len(keys)
    full, view = full_index_of_records(ins, len(cams))
    it = ins["inst_tile"].cpu().numpy().view(np.uint32).astype(np.uint64)
    ir = ins["inst_record"].cpu().numpy().view(np.uint32).astype(np.int64)
    dk = ins["depth_key"].cpu().numpy().view(np.uint32).astype(np.uint64)
    assert np.array_equal((it << np.uint64(32)) | dk[ir], keys)
    assert np.array_equal(view[ir] * sc.n + full[ir], vals)
    assert np.array_equal(ins["ranges"].cpu().numpy().view(np.uint32), ranges)


@pytest.mark.parametrize("sizes", [[(128, 128)], [(100, 75)], [(128, 128), (72, 40)]])
def test_binning_bit_exact(rz, sizes):
    sc = scenes.tiny_scene(800, seed_salt=4)
    cams = [scenes.tiny_camera(w, h) for w, h in sizes]
    fr = gpu_forward(rz, sc, cams)
    ins = rz.inspect(fr)
    keys, vals, ranges = _oracle_bins(sc, cams)
    V = len(cams)
    M = ins["info"]["instances"]
    assert M == len(keys)
    full, view = full_index_of_records(ins, V)
    it = ins["inst_tile"].cpu().numpy().view(np.uint32).astype(np.uint64)
    ir = ins["inst_record"].cpu().numpy().view(np.uint32).astype(np.int64)
    dk = ins["depth_key"].cpu().numpy().view(np.uint32).astype(np.uint64)
    gkeys = (it << np.uint64(32)) | dk[ir]
    gvals = view[ir] * sc.n + full[ir]
    assert np.array_equal(gkeys, keys)
    assert np.array_equal(gvals, vals)
    gr = ins["ranges"].cpu().numpy().view(np.uint32)
    # empty tiles are (0, 0) on the GPU and in the oracle
    assert np.array_equal(gr, ranges)


def test_binning_bit_exact_wide_sort_tiles(rz):
    """A workspace sized for 2^24 + 5 instances: the tile sort takes its large-sort
    tiles (4096 items per block) while the frame holds a few thousand instances. The
    lists stay bit-exact."""
    import ctypes
    from paper_2503_01199_amd import _lib as L
    from paper_2503_01199_amd.raster import SceneTensors, Workspace, camera_struct
    sc = scenes.tiny_scene(800, seed_salt=4)
    cams = [scenes.tiny_camera(128, 128), scenes.tiny_camera(72, 40)]
    st = SceneTensors.from_scene(sc, rz.device)
    cs = (L.GsrCamera * len(cams))(*[camera_struct(c) for c in cams])
    nbytes = ctypes.c_size_t()
    rz._check(rz.lib.gsr_workspace_size(rz.ctx, ctypes.byref(st.struct()), cs, len(cams),
                                        ctypes.byref(rz.options(L.GSR_FP32, True, True, False)), (1 << 24) + 5,
                                        ctypes.byref(nbytes)), "gsr_workspace_size")
    ws = Workspace(rz.device)
    ws.ensure(nbytes.value)
    print("wide tile sort: workspace %d bytes" % nbytes.value, flush=True)
    fr = rz.forward(st, cams, workspace=ws)
    torch.cuda.synchronize()
    ins = rz.inspect(fr)
    keys, vals, ranges = _oracle_bins(sc, cams)
    assert ins["info"]["instances"] == len(keys)
    full, view = full_index_of_records(ins, len(cams))
    it = ins["inst_tile"].cpu().numpy().view(np.uint32).astype(np.uint64)
    ir = ins["inst_record"].cpu().numpy().view(np.uint32).astype(np.int64)
    dk = ins["depth_key"].cpu().numpy().view(np.uint32).astype(np.uint64)
    assert np.array_equal((it << np.uint64(32)) | dk[ir], keys)
    assert np.array_equal(view[ir] * sc.n + full[ir], vals)
    assert np.array_equal(ins["ranges"].cpu().numpy().view(np.uint32), ranges)


def test_pixel_state_matches_tiled_oracle(rz):
    sc, cam = scenes.tiny_scene(), scenes.tiny_camera()
    sc.opacity_logits[:] = sc.opacity_logits + 2.0  # reach the T stop on many pixels
    fr = gpu_forward(rz, sc, [cam])
    ref = check_image(fr, sc, cam, what="dense tiny")
    ins = rz.inspect(fr)
    keep = ~ref["fragile"].ravel()
    last = ins["pixel_last"].cpu().numpy().view(np.uint32)
    assert np.array_equal(last[keep], ref["n_contrib"].ravel()[keep])
    T = ins["pixel_T"].cpu().numpy()
    assert np.abs(T - ref["T"].ravel())[keep].max() < 1e-5
    assert (T >= 1e-4).all() and (T <= 1).all()
    assert (ref["T"] < 1e-3).sum() > 50


@pytest.mark.parametrize("size", [(128, 128), (100, 75)])
def test_split_tiles_match_oracle(rz, size):
    """6,000 Gaussians on a small image: most tile lists exceed 256 entries, so the
    longest (at most a quarter of the tiles) are rastered as four 16x4 band items.
    The image and the per-pixel state (T, last blended position) match the oracle
    as for whole tiles; at 100x75 the split tiles include the ragged bottom row,
    whose last band lies wholly below the image."""
    sc = scenes.tiny_scene(6000, seed_salt=9)
    cam = scenes.tiny_camera(*size)
    fr = gpu_forward(rz, sc, [cam])
    ref = check_image(fr, sc, cam, what="split tiles %dx%d" % size)
    ins = rz.inspect(fr)
    _, _, ranges = _oracle_bins(sc, [cam])
    lens = ranges[:, 1].astype(np.int64) - ranges[:, 0]
    cap = -(-len(lens) // 4)
    expect, expect_bwd = min(int((lens > 256).sum()), cap), min(int((lens > 512).sum()), cap)
    print("split tiles %d of %d (longest list %d)" % (ins["info"]["split_tiles"], len(lens), lens.max()))
    assert ins["info"]["split_tiles"] == expect and expect > 0
    assert ins["info"]["split_tiles_bwd"] == expect_bwd
    keep = ~ref["fragile"].ravel()
    last = ins["pixel_last"].cpu().numpy().view(np.uint32)
    assert np.array_equal(last[keep], ref["n_contrib"].ravel()[keep])
    T = ins["pixel_T"].cpu().numpy()
    assert np.abs(T - ref["T"].ravel())[keep].max() < 1e-5


def test_ragged_and_batched_views_equal_single(rz):
    sc = scenes.tiny_scene(700, seed_salt=6)
    cams = [scenes.tiny_camera(100, 75), scenes.tiny_camera(37, 53), scenes.tiny_camera(128, 128)]
    fr = gpu_forward(rz, sc, cams)
    for v, cam in enumerate(cams):
        check_image(fr, sc, cam, v=v, what="view %d" % v)
        single = gpu_forward(rz, sc, [cam])
        assert torch.equal(single.images[0], fr.images[v])


def test_empty_and_invisible_scenes_render_background(rz):
    cam = scenes.tiny_camera(40, 24)
    cam.bg = (0.25, 0.5, 0.75)
    empty = scenes.tiny_scene(0)
    fr = gpu_forward(rz, empty, [cam])
    img = fr.images[0].cpu().numpy()
    for ch in range(3):
        assert np.all(img[ch] == np.float32(cam.bg[ch]))
    behind = scenes.tiny_scene(300)
    behind.means[:, 2] = -behind.means[:, 2]  # all behind the camera
    fr = gpu_forward(rz, behind, [cam])
    assert fr.info["instances"] == 0
    assert np.all(fr.images[0].cpu().numpy()[2] == np.float32(0.75))


def test_cluster_cull_is_neutral_and_conservative(rz):
    sc = scenes.spheres_planes_scene(30_000, seed_salt=1)
    # Morton order makes clusters compact so the cull has something to remove
    codes, perm = orc.morton(sc.means)
    sc = sc.permuted(perm)
    cam = scenes.spheres_planes_camera()
    on = gpu_forward(rz, sc, [cam], cull=True)
    off = gpu_forward(rz, sc, [cam], cull=False)
    assert torch.equal(on.images[0], off.images[0])
    ins = rz.inspect(on)
    vis = ins["cluster_visible"].cpu().numpy()[: on.info["clusters"]]
    print("visible clusters %d of %d" % (vis.sum(), vis.size))
    assert vis.sum() < vis.size  # something was culled
    pp = orc.preprocess(sc, cam)
    for c in np.nonzero(vis == 0)[0]:
        assert pp["tiles"][c * 128:(c + 1) * 128].sum() == 0
    check_image(on, sc, cam, what="spheres 30k")


def test_spheres_scene_full_size(rz):
    """200k Gaussians, SH degree 3, 800x800, Morton-ordered, cull on: image and binning."""
    sc = scenes.spheres_planes_scene()
    _, perm = orc.morton(sc.means)
    sc = sc.permuted(perm)
    cam = scenes.spheres_planes_camera()
    fr = gpu_forward(rz, sc, [cam])
    check_image(fr, sc, cam, what="spheres 200k")
    ins = rz.inspect(fr)
    keys, vals, ranges = _oracle_bins(sc, [cam])
    assert ins["info"]["instances"] == len(keys)
    full, _ = full_index_of_records(ins, 1)
    it = ins["inst_tile"].cpu().numpy().view(np.uint32).astype(np.uint64)
    ir = ins["inst_record"].cpu().numpy().view(np.uint32).astype(np.int64)
    dk = ins["depth_key"].cpu().numpy().view(np.uint32).astype(np.uint64)
    assert np.array_equal((it << np.uint64(32)) | dk[ir], keys)
    assert np.array_equal(full[ir], vals)
    assert np.array_equal(ins["ranges"].cpu().numpy().view(np.uint32), ranges)


def test_views_beyond_one_argument_chunk(rz):
    """20 views of ragged sizes: the view table is uploaded in kernel-argument chunks
    of 16, so views 16..19 come from a second chunk."""
    sc = scenes.tiny_scene(500, seed_salt=8)
    cams = [scenes.tiny_camera(40 + 3 * k, 30 + 2 * k) for k in range(20)]
    fr = gpu_forward(rz, sc, cams)
    ins = rz.inspect(fr)
    keys, vals, ranges = _oracle_bins(sc, cams)
    assert ins["info"]["instances"] == len(keys)
    full, view = full_index_of_records(ins, len(cams))
    it = ins["inst_tile"].cpu().numpy().view(np.uint32).astype(np.uint64)
    ir = ins["inst_record"].cpu().numpy().view(np.uint32).astype(np.int64)
    dk = ins["depth_key"].cpu().numpy().view(np.uint32).astype(np.uint64)
    assert np.array_equal((it << np.uint64(32)) | dk[ir], keys)
    assert np.array_equal(view[ir] * sc.n + full[ir], vals)
    for v in (0, 15, 16, 19):
        check_image(fr, sc, cams[v], v=v, what="view %d of 20" % v)


@pytest.mark.parametrize("large", [False, True])
def test_instance_overflow_keeps_a_depth_prefix_and_reports(rz, large):
    """A workspace that holds about half of the frame's instances: the forward cuts
    the list at the capacity, every tile keeps a prefix of its full list, and the
    frame check reports the workspace the frame needs; after growing, the frame is
    whole again. With large footprints the cut can fall inside a record that a whole
    wave emits."""
    import ctypes
    from paper_2503_01199_amd import _lib as L
    from paper_2503_01199_amd.raster import SceneTensors, Workspace, camera_struct
    sc = _large_footprint_scene() if large else scenes.tiny_scene()
    cam = scenes.tiny_camera()
    st = SceneTensors.from_scene(sc, rz.device)
    full = rz.forward(st, [cam], workspace=Workspace(rz.device))
    fins = rz.inspect(full)
    M = fins["info"]["instances"]
    assert M > 1000
    cams = (L.GsrCamera * 1)(camera_struct(cam))
    nbytes = ctypes.c_size_t()
    sct = st.struct()
    assert rz.lib.gsr_workspace_size(rz.ctx, ctypes.byref(sct), cams, 1, ctypes.byref(full.opts), M // 2,
                                     ctypes.byref(nbytes)) == L.GSR_OK
    ws = Workspace(rz.device)
    ws.ensure(nbytes.value)
    print("overflow case: M=%d, workspace for %d" % (M, M // 2), flush=True)
    cut = rz.forward(st, [cam], workspace=ws, check=False)
    with pytest.raises(L.GsrError, match="WORKSPACE_TOO_SMALL"):
        rz.check_frame(cut)
    assert rz.lib.gsr_required_workspace(rz.ctx) > nbytes.value
    ins = rz.inspect(cut, allow_overflow=True)
    kept = ins["info"]["kept"]
    assert ins["info"]["instances"] == M and M // 2 <= kept < M
    fr_r = fins["ranges"].cpu().numpy().view(np.uint32).astype(np.int64)
    cr = ins["ranges"].cpu().numpy().view(np.uint32).astype(np.int64)
    fr_rec = fins["inst_record"].cpu().numpy().view(np.uint32)
    c_rec = ins["inst_record"].cpu().numpy().view(np.uint32)
    assert (cr[:, 1] - cr[:, 0]).sum() == kept
    for t in range(cr.shape[0]):
        n_cut = cr[t, 1] - cr[t, 0]
        assert n_cut <= fr_r[t, 1] - fr_r[t, 0]
        if n_cut:
            assert np.array_equal(c_rec[cr[t, 0]:cr[t, 1]], fr_rec[fr_r[t, 0]:fr_r[t, 0] + n_cut])
    again = rz.forward(st, [cam], workspace=ws)
    assert again.info["instances"] == M
    assert torch.equal(again.images[0], full.images[0])
