"""The deterministic backward (gsr_options.deterministic): per-tile gradient sums
added as 64-bit fixed-point integers at one scale shared by the frame's tiles.

Integer addition is associative, so the result cannot depend on the order in
which tiles finish: repeated backward passes and the same frame rendered in a batch
of other frames must give bitwise identical gradients and statistic. The scale
follows the upstream gradient: with 2^E the power of two above max |dL/dI|, each
per-tile sum is rounded to a multiple of 2^(E-32) (the statistic's square sum to
2^(2E-32)), which moves a gradient by at most (tiles touched) x 2^(E-33) from the
FP32 sum, far inside the 1e-3 parity bar at any loss scale; the tests below apply
that bar against the FP64 oracle, including with a mean-reduced loss (upstream
gradients of order 1/(3HW))."""
import numpy as np
import pytest
import torch

import oracle as orc
from helpers import ensure_built
from paper_2503_01199_amd import scenes
from parity import GROUPS, compare, oracle_sum, upstream

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rz():
    ensure_built()
    from paper_2503_01199_amd.raster import Rasterizer
    return Rasterizer(0)


def _backward(rz, fr, gI, stats=True):
    from paper_2503_01199_amd.raster import new_stats
    st = new_stats(fr.scene.n, rz.device) if stats else None
    g = rz.backward(fr, [torch.as_tensor(x, device=rz.device) for x in gI], stats=st)
    torch.cuda.synchronize()
    out = {k: v.cpu().numpy().copy() for k, v in g.items()}
    if st is not None:
        out.update({"stat_" + k: v.cpu().numpy().copy() for k, v in st.items()})
    return out


@pytest.mark.parametrize("which", ["tiny", "split", "mean-loss", "room-mean-loss"])
def test_deterministic_gradients_match_oracle(rz, which):
    """Gradients, S, M and C against the oracle. mean-loss: the upstream gradient of
    the L1 loss divided by 3HW (as a mean-reduced loss gives), so per-tile sums are
    ~1e-7 and the statistic's square sums ~1e-12; room-mean-loss: the same scale at
    the room's 1600x1064 (2e-7 per pixel) on its centre crop."""
    from paper_2503_01199_amd.raster import SceneTensors, Workspace
    if which == "tiny":
        sc, cam = scenes.tiny_scene(), scenes.tiny_camera()
    elif which == "room-mean-loss":
        sc, cam = scenes.tiny_scene(6000, seed_salt=9), scenes.tiny_camera()
        cam = scenes.Camera(1600, 1064, cam.fx, cam.fy, cam.cx, cam.cy, cam.R, cam.t, cam.near, cam.bg)
    else:  # long lists: split tiles in both rasters
        sc, cam = scenes.tiny_scene(6000, seed_salt=9), scenes.tiny_camera()
    gI, _ = upstream(sc, [cam])
    if which in ("mean-loss", "room-mean-loss"):
        gI = [(g / np.float32(3 * cam.width * cam.height)).astype(np.float32) for g in gI]
        print("upstream max |dL/dI| %.3g" % max(float(np.abs(g).max()) for g in gI))
    print("deterministic backward %s n=%d" % (which, sc.n), flush=True)
    fr = rz.forward(SceneTensors.from_scene(sc, rz.device), [cam], workspace=Workspace(rz.device), deterministic=True)
    out = _backward(rz, fr, gI)
    ref = oracle_sum(sc, [cam], gI)
    grads = {k: out[k] for k in GROUPS}
    stats = {k: out["stat_" + k] for k in ("S", "M", "C")}
    if which in ("mean-loss", "room-mean-loss"):
        # per-tile square sums far below a fixed 2^-32 step, which rounded them to 0
        print("oracle S: max %.3g" % np.abs(ref["S"]).max())
        assert max(float(np.abs(g).max()) for g in gI) < 1e-4
    compare(grads, stats, ref, "deterministic %s" % which, logits=sc.opacity_logits)


def test_repeated_backward_is_bitwise_identical(rz):
    """30k Gaussians on spheres and planes, 320x240: many tiles add into the same
    records. Three deterministic backward passes agree bit for bit; the FP32-atomic
    passes are reported (they may differ in the last bits)."""
    from paper_2503_01199_amd.raster import SceneTensors, Workspace
    sc = scenes.spheres_planes_scene(30_000, seed_salt=5)
    _, perm = orc.morton(sc.means)
    sc = sc.permuted(perm)
    cam = scenes.orbit_camera(30.0, 15.0, radius=5.0, width=320, height=240)
    w, _ = scenes.l1_weights((3, cam.height, cam.width), config=0, salt=4)
    gI = [w * np.sign(np.random.default_rng(4).standard_normal(w.shape)).astype(np.float32)]
    st = SceneTensors.from_scene(sc, rz.device)
    print("repeated deterministic backward n=%d" % sc.n, flush=True)
    fr = rz.forward(st, [cam], workspace=Workspace(rz.device), deterministic=True)
    runs = [_backward(rz, fr, gI) for _ in range(3)]
    for r in runs[1:]:
        for k in runs[0]:
            assert np.array_equal(r[k], runs[0][k]), k
    ff = rz.forward(st, [cam], workspace=Workspace(rz.device))
    fl = [_backward(rz, ff, gI) for _ in range(3)]
    differ = sum(int(not np.array_equal(r[k], fl[0][k])) for r in fl[1:] for k in fl[0])
    print("FP32 atomics: %d of %d arrays differ between repeated passes" % (differ, 2 * len(fl[0])))
    for k in GROUPS:  # the two reductions agree to FP32 rounding of the per-tile sums
        scale = float(np.abs(fl[0][k]).max()) + 1e-30
        assert float(np.abs(runs[0][k] - fl[0][k]).max()) <= 1e-5 * scale, k


def test_batched_frame_backward_is_bitwise_identical(rz):
    """A frame rastered inside a batch of other frames and the same frame alone:
    identical gradients, bit for bit."""
    from paper_2503_01199_amd.raster import SceneTensors, Workspace
    a = SceneTensors.from_scene(scenes.tiny_scene(6000, seed_salt=9), rz.device)
    b = SceneTensors.from_scene(scenes.spheres_planes_scene(20_000, seed_salt=2), rz.device)
    cam_a = scenes.tiny_camera(100, 75)
    cam_b = scenes.orbit_camera(10.0, 5.0, radius=7.0, width=200, height=150)
    gI = [np.random.default_rng(8).uniform(-1, 1, (3, cam_a.height, cam_a.width)).astype(np.float32)]
    print("batched deterministic backward", flush=True)
    frames = [rz.prepare(b, [cam_b], workspace=Workspace(rz.device), deterministic=True),
              rz.prepare(a, [cam_a], workspace=Workspace(rz.device), deterministic=True)]
    rz.raster_batch(frames)
    torch.cuda.synchronize()
    rz.check_frame(frames[1])
    g_batch = _backward(rz, frames[1], gI)
    alone = rz.forward(a, [cam_a], workspace=Workspace(rz.device), deterministic=True)
    g_alone = _backward(rz, alone, gI)
    for k in g_alone:
        assert np.array_equal(g_batch[k], g_alone[k]), k


def test_backward_must_match_the_forward_mode(rz):
    from paper_2503_01199_amd import _lib as L
    from paper_2503_01199_amd.raster import SceneTensors, Workspace
    sc, cam = scenes.tiny_scene(), scenes.tiny_camera()
    fr = rz.forward(SceneTensors.from_scene(sc, rz.device), [cam], workspace=Workspace(rz.device))
    fr.opts.deterministic = 1  # the frame was rendered without the fixed-point buffer
    with pytest.raises(L.GsrError):
        rz.backward(fr, [torch.zeros((3, cam.height, cam.width), device=rz.device)])


@pytest.mark.parametrize("split", [(0xffffffff, 0xffffffff), (64, 128), (0, 0)])
def test_raster_schedule_changes_nothing_but_time(rz, split):
    """The split thresholds of the raster schedules (never, low, default) leave the
    image bitwise unchanged and split the expected tiles: the longest min(#lists
    above the threshold, T/4). The deterministic gradients are bitwise unchanged
    while the backward's schedule is; a tile walked as two halves adds two
    separately rounded sums, which moves a gradient by FP32 rounding only."""
    from paper_2503_01199_amd.raster import SceneTensors, Workspace
    sc, cam = scenes.tiny_scene(6000, seed_salt=9), scenes.tiny_camera()
    st = SceneTensors.from_scene(sc, rz.device)
    gI = [np.random.default_rng(2).uniform(-1, 1, (3, cam.height, cam.width)).astype(np.float32)]
    ref = rz.forward(st, [cam], workspace=Workspace(rz.device), deterministic=True)
    g_ref = _backward(rz, ref, gI)
    bwd_ref = rz.inspect(ref)["info"]["split_tiles_bwd"]
    print("schedule split=%s" % (split,), flush=True)
    rz.set_raster_split(*split)
    try:
        fr = rz.forward(st, [cam], workspace=Workspace(rz.device), deterministic=True)
        g = _backward(rz, fr, gI)
        ins = rz.inspect(fr)
        # where the quarter cap cuts through tiles of equal length, the split ones are
        # picked by index: a second frame splits the same tiles, so it is bitwise equal
        g2 = _backward(rz, rz.forward(st, [cam], workspace=Workspace(rz.device), deterministic=True), gI)
    finally:
        rz.set_raster_split(0, 0)
    for k in g:
        assert np.array_equal(g[k], g2[k]), k
    assert torch.equal(fr.images[0], ref.images[0])
    for k in g_ref:
        if ins["info"]["split_tiles_bwd"] == bwd_ref:
            assert np.array_equal(g[k], g_ref[k]), k
        else:
            scale = float(np.abs(g_ref[k]).max()) + 1e-30
            assert float(np.abs(g[k].astype(np.float64) - g_ref[k]).max()) <= 1e-5 * scale, k
    lens = np.diff(ins["ranges"].cpu().numpy().astype(np.int64), axis=1).ravel()
    cap = (lens.size + 3) // 4
    f_len = 256 if split[0] == 0 else split[0]
    b_len = 512 if split[1] == 0 else split[1]
    assert ins["info"]["split_tiles"] == min(int((lens > f_len).sum()), cap)
    assert ins["info"]["split_tiles_bwd"] == min(int((lens > b_len).sum()), cap)


def test_autograd_deterministic_gradients_repeat(rz):
    """rasterize(..., deterministic=True): two loss.backward() calls leave the same
    gradient bits in the parameter tensors."""
    from paper_2503_01199_amd.autograd import rasterize
    sc = scenes.tiny_scene(3000, seed_salt=3)
    cams = [scenes.tiny_camera(96, 80), scenes.tiny_camera(64, 64)]
    w = [torch.as_tensor(np.random.default_rng(v).uniform(-1, 1, (3, c.height, c.width)).astype(np.float32),
                         device=rz.device) for v, c in enumerate(cams)]
    runs = []
    print("deterministic autograd n=%d" % sc.n, flush=True)
    for _ in range(2):
        params = [torch.as_tensor(a, device=rz.device).requires_grad_(True) for a in sc.arrays()]
        imgs = rasterize(*params, cams, sc.sh_degree, rasterizer=rz, deterministic=True)
        sum((img * wi).sum() for img, wi in zip(imgs, w)).backward()
        runs.append([p.grad.detach().clone() for p in params])
    for a, b in zip(*runs):
        assert torch.equal(a, b)
