"""Batched raster and serving on the GPU: a frame rendered inside a batch of frames
of other scenes and sizes, or served in a mix of concurrent requests, equals the
same frame rendered alone, bit for bit (tiles are independent and the forward has
no atomics)."""
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


@pytest.fixture(scope="module")
def small_scenes(rz):
    from paper_2503_01199_amd.raster import SceneTensors
    a = SceneTensors.from_scene(scenes.tiny_scene(1024), rz.device)
    b = SceneTensors.from_scene(scenes.spheres_planes_scene(30_000, seed_salt=5), rz.device)
    perm, _ = rz.morton_order(b.means)
    b = SceneTensors(*rz.apply_permutation(perm, list(b.tensors())), b.sh_degree)
    d = SceneTensors.from_scene(scenes.tiny_scene(6000, seed_salt=9), rz.device)  # lists long enough to split
    return {"tiny": a, "spheres": b, "dense": d}


@pytest.mark.parametrize("precision", ["fp32", "fp16"])
def test_batched_raster_equals_single_frames(rz, small_scenes, precision):
    from paper_2503_01199_amd import _lib as L
    from paper_2503_01199_amd.raster import Workspace
    prec = L.GSR_FP16_BLEND if precision == "fp16" else L.GSR_FP32
    jobs = [("tiny", [scenes.tiny_camera()]),
            ("spheres", [scenes.orbit_camera(20.0, 5.0, radius=7.0, width=200, height=150)]),
            ("tiny", [scenes.tiny_camera(100, 75), scenes.tiny_camera(37, 53)]),
            ("spheres", [scenes.orbit_camera(200.0, 20.0, radius=7.0, width=320, height=240)])]
    print("batch of %d frames, %s" % (len(jobs), precision), flush=True)
    frames = [rz.prepare(small_scenes[n], cams, workspace=Workspace(rz.device)) for n, cams in jobs]
    imgs = rz.raster_batch(frames, precision=prec)
    torch.cuda.synchronize()
    for (n, cams), im, fr in zip(jobs, imgs, frames):
        rz.check_frame(fr)
        alone = rz.forward(small_scenes[n], cams, precision=prec, workspace=Workspace(rz.device))
        for a, b in zip(alone.images, im):
            assert torch.equal(a, b)
    # a batched frame can be differentiated like any other
    fr = frames[1]
    dl = [torch.ones_like(t) for t in fr.images]
    g_batch = {k: v.clone() for k, v in rz.backward(fr, dl).items()}
    alone = rz.forward(small_scenes["spheres"], jobs[1][1], precision=prec, workspace=Workspace(rz.device))
    g_alone = rz.backward(alone, dl)
    for k in g_batch:  # equal up to the order of the float atomics
        scale = float(g_alone[k].abs().max().item()) + 1e-30
        assert float((g_batch[k] - g_alone[k]).abs().max().item()) <= 1e-5 * scale, k


def test_batched_split_tiles_equal_single_frames(rz, small_scenes):
    """A batch caps its split tiles over all its frames, so a dense frame's tiles can
    be split differently in the batch and alone; its image must not change (a band
    item evaluates its pixels exactly as the whole-tile walk does)."""
    from paper_2503_01199_amd.raster import Workspace
    jobs = [("dense", [scenes.tiny_camera()]), ("spheres", [scenes.orbit_camera(20.0, 5.0, radius=7.0, width=200,
                                                                                  height=150)]),
            ("dense", [scenes.tiny_camera(100, 75)])]
    frames = [rz.prepare(small_scenes[n], cams, workspace=Workspace(rz.device)) for n, cams in jobs]
    imgs = rz.raster_batch(frames)
    torch.cuda.synchronize()
    for (n, cams), im in zip(jobs, imgs):
        alone = rz.forward(small_scenes[n], cams, workspace=Workspace(rz.device))
        if n == "dense":
            assert rz.inspect(alone)["info"]["split_tiles"] > 0
        for a, b in zip(alone.images, im):
            assert torch.equal(a, b)


def test_served_images_equal_rendering_alone(rz, small_scenes):
    from paper_2503_01199_amd import _lib as L
    from paper_2503_01199_amd.raster import Workspace
    from paper_2503_01199_amd.serve import GpuExecutor, Request, Scheduler
    ex = GpuExecutor(rz, small_scenes, slots=6)
    for name in small_scenes:
        ex.calibrate(name, scenes.orbit_camera(0.0, 10.0, radius=7.0, width=256, height=256))
    rng = np.random.default_rng(5)
    sizes = [(256, 256), (512, 512), (320, 180), (96, 64)]
    reqs = []
    for i in range(24):
        w, h = sizes[i % 4]
        name = "spheres" if i % 3 else "tiny"
        cam = (scenes.orbit_camera(float(rng.uniform(0, 360)), float(rng.uniform(-10, 30)), radius=7.0, width=w,
                                   height=h) if name == "spheres" else scenes.tiny_camera(w, h))
        reqs.append(Request(i, name, cam, arrival=i * 2e-4))
    print("serving %d requests" % len(reqs), flush=True)
    st = Scheduler(ex, budget_bytes=1 << 30, slots=6).run(reqs)
    torch.cuda.synchronize()
    print("served: %s" % st.summary())
    assert len(st.latencies) == len(reqs) and st.rejected == 0
    assert max(st.batch_sizes) > 1  # requests shared launches
    for r in reqs:
        alone = rz.forward(small_scenes[r.scene], [r.camera], precision=L.GSR_FP16_BLEND,
                           workspace=Workspace(rz.device))
        assert torch.equal(alone.images[0], r.images[0]), r.rid


def test_tiny_budget_serves_one_request_at_a_time(rz, small_scenes):
    from paper_2503_01199_amd.serve import GpuExecutor, Request, Scheduler
    ex = GpuExecutor(rz, small_scenes, slots=4)
    for name in small_scenes:
        ex.calibrate(name, scenes.orbit_camera(0.0, 10.0, radius=7.0, width=256, height=256))
    reqs = [Request(i, "spheres", scenes.orbit_camera(15.0 * i, 10.0, radius=7.0, width=256, height=256), 0.0)
            for i in range(8)]
    need = max(ex.bytes_needed(r) for r in reqs)
    st = Scheduler(ex, budget_bytes=int(need * 1.2), slots=4).run(reqs)
    print("tiny budget: %s" % st.summary())
    assert len(st.latencies) == 8
    assert st.max_bytes_in_use <= int(need * 1.2)
    assert max(st.batch_sizes) == 1 and max(st.admission_waits) > 0
