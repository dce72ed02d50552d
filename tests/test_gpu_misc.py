"""GPU: Morton order, permutation, loss gradient, autograd, error paths."""
import numpy as np
import pytest
import torch

import oracle as orc
from helpers import ensure_built
from paper_2503_01199_amd import scenes

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rz():
    ensure_built()
    from paper_2503_01199_amd.raster import Rasterizer
    return Rasterizer(0)


@pytest.mark.parametrize("n", [1, 1000, 200_003])
def test_morton_codes_and_order_bit_exact(rz, n):
    sc = scenes.spheres_planes_scene(max(n, 2), seed_salt=3) if n > 1 else scenes.tiny_scene(1)
    means = sc.means[:n].copy()
    means[n // 3: n // 3 + min(5, n // 3)] = means[0]  # exact duplicates exercise the stable order
    print("morton n=%d" % n, flush=True)
    perm, codes = rz.morton_order(torch.as_tensor(means, device=rz.device))
    ref_codes, ref_perm = orc.morton(means)
    assert np.array_equal(codes.cpu().numpy().view(np.uint64), ref_codes)
    assert np.array_equal(perm.cpu().numpy(), ref_perm)


def test_morton_order_wide_sort_tiles(rz):
    """2^24 + 3 points: the 64-bit code sort takes its large-sort tiles (4096 items
    per block, 8 passes). Points on a coarse grid, so many codes repeat and the
    stable order of equal codes is exercised in every pass."""
    n = (1 << 24) + 3
    rng = np.random.default_rng(11)
    means = (rng.integers(0, 300, size=(n, 3)) * np.float32(0.01) - np.float32(1.5)).astype(np.float32)
    print("morton n=%d" % n, flush=True)
    perm, codes = rz.morton_order(torch.as_tensor(means, device=rz.device))
    ref_codes, ref_perm = orc.morton(means)
    assert np.array_equal(codes.cpu().numpy().view(np.uint64), ref_codes)
    assert np.array_equal(perm.cpu().numpy(), ref_perm)


def test_morton_degenerate_axis(rz):
    m = np.zeros((300, 3), np.float32)
    m[:, 0] = np.linspace(-1, 1, 300)  # y and z constant
    perm, codes = rz.morton_order(torch.as_tensor(m, device=rz.device))
    ref_codes, ref_perm = orc.morton(m)
    assert np.array_equal(codes.cpu().numpy().view(np.uint64), ref_codes)
    assert np.array_equal(perm.cpu().numpy(), ref_perm)


def test_permutation_is_neutral_for_the_image(rz):
    """Reordering the scene does not change the image when no two Gaussians share a
    depth key (ties legitimately fall back to the caller's order)."""
    from paper_2503_01199_amd.raster import SceneTensors, Workspace
    sc = scenes.tiny_scene(3000, seed_salt=0)
    cam = scenes.tiny_camera()
    st = SceneTensors.from_scene(sc, rz.device)
    perm, _ = rz.morton_order(st.means)
    arrs = rz.apply_permutation(perm, list(st.tensors()))
    ref = [a[perm] for a in st.tensors()]
    for a, b in zip(arrs, ref):
        assert torch.equal(a, b)
    a = rz.forward(st, [cam], workspace=Workspace(rz.device))
    b = rz.forward(SceneTensors(*arrs, st.sh_degree), [cam], workspace=Workspace(rz.device))
    dk = rz.inspect(a)["depth_key"].cpu().numpy()
    valid = dk[dk != -1]
    assert np.unique(valid).size == valid.size  # the premise: no depth ties
    assert torch.equal(a.images[0], b.images[0])


def test_l1_gradient_kernel(rz):
    rng = np.random.default_rng(5)
    for n in (3 * 37 * 53, 4 * 1000 + 3):
        img, w, gt = (rng.uniform(0, 1, n).astype(np.float32) for _ in range(3))
        gt[::7] = img[::7]  # ties give 0
        t = lambda a: torch.as_tensor(a, device=rz.device)  # noqa: E731
        out = rz.l1_grad(t(img), t(w), t(gt)).cpu().numpy()
        assert np.array_equal(out, (w * np.sign(img - gt)).astype(np.float32))


def test_workspace_grows_and_errors_are_reported(rz):
    from paper_2503_01199_amd import _lib as L
    from paper_2503_01199_amd.raster import SceneTensors, Workspace
    sc, cam = scenes.tiny_scene(), scenes.tiny_camera()
    st = SceneTensors.from_scene(sc, rz.device)
    ws = Workspace(rz.device)
    ws.ensure(1 << 16)  # far too small: the binding must grow it from the reported size
    fr = rz.forward(st, [cam], workspace=ws)
    assert ws.nbytes > (1 << 16) and fr.info["instances"] > 0
    # invalid arguments come back as GSR_ERR_INVALID_ARG with a message
    with pytest.raises(L.GsrError, match="INVALID_ARG"):
        bad = SceneTensors(st.means, st.log_scales, st.quats, st.opacity_logits, st.sh, 4)
        rz.forward(bad, [cam], workspace=Workspace(rz.device))
    with pytest.raises(L.GsrError, match="INVALID_ARG"):
        rz.forward(st, [cam], precision=7, workspace=Workspace(rz.device))
    # backward before any forward on a workspace is rejected
    from paper_2503_01199_amd.raster import Frame
    fake = Frame(st, [cam], fr.cam_structs, fr.opts, Workspace(rz.device), fr.images, {})
    fake.workspace.ensure(1024)
    with pytest.raises(L.GsrError, match="INVALID_ARG"):
        rz.backward(fake, [torch.zeros((3, cam.height, cam.width), device=rz.device)])


def test_stage_times_are_recorded(rz):
    from paper_2503_01199_amd.raster import SceneTensors, Workspace
    sc, cam = scenes.tiny_scene(), scenes.tiny_camera()
    st = SceneTensors.from_scene(sc, rz.device)
    rz.set_profiling(True)
    fr = rz.forward(st, [cam], workspace=Workspace(rz.device))
    dl = [torch.ones((3, cam.height, cam.width), device=rz.device)]
    g1 = {k: v.clone() for k, v in rz.backward(fr, dl).items()}
    t = rz.stage_times()
    # the forward clears the gradient rows of its records, so the first backward
    # has no clearing stage; a repeated backward clears them itself
    assert t["zero_grad"] == -1.0 and all(v >= 0 for k, v in t.items() if k != "zero_grad"), t
    g2 = rz.backward(fr, dl)
    t = rz.stage_times()
    rz.set_profiling(False)
    assert t["zero_grad"] >= 0, t
    for k in g1:  # equal up to the order of the float atomics
        scale = float(g1[k].abs().max().item()) + 1e-30
        assert float((g1[k] - g2[k]).abs().max().item()) <= 1e-5 * scale, k


def _loss64(images, weights):
    return sum(float((img.double() * w.double()).sum().item()) for img, w in zip(images, weights))


def test_autograd_function_matches_oracle_and_directional_differences(rz):
    from paper_2503_01199_amd.autograd import rasterize
    sc = scenes.tiny_scene(800, seed_salt=9)
    cams = [scenes.tiny_camera(96, 80), scenes.tiny_camera(64, 64)]
    dev = rz.device
    params = [torch.as_tensor(a, device=dev).requires_grad_(True) for a in sc.arrays()]
    rng = np.random.default_rng(0)
    weights = [torch.as_tensor(rng.uniform(-1, 1, (3, c.height, c.width)).astype(np.float32), device=dev)
               for c in cams]
    imgs = rasterize(*params, cams, sc.sh_degree, rasterizer=rz)
    loss = sum((img * w).sum() for img, w in zip(imgs, weights))
    loss.backward()
    g = [p.grad.detach().cpu().numpy().astype(np.float64) for p in params]
    # the autograd gradient is the library's backward: compare with the oracle
    ref = None
    for cam, w in zip(cams, weights):
        b = orc.backward(sc, cam, w.cpu().numpy().astype(np.float64), mode=1)
        ref = b if ref is None else {k: ref[k] + b[k] for k in ("means", "log_scales", "quats",
                                                                   "opacity_logits", "sh")}
    for k, gk in zip(("means", "log_scales", "quats", "opacity_logits", "sh"), g):
        err = np.abs(gk - ref[k]).max() / np.abs(ref[k]).max()
        print("autograd vs oracle %-15s %.3g" % (k, err))
        assert err < 1e-3
    # central differences of the FP32 forward (loss summed in FP64), one scalar at a
    # time, step 3e-3 relative (the FP32 forward's rounding of the exponent, which the
    # scanline extrapolates up to 6 rows from the strip's anchor, sets a noise floor of
    # ~1e-7 / h). A probe whose stencil changes any pixel's blended set (the alpha
    # cutoff makes the loss discontinuous at footprint edges) is replaced by another:
    # the tile lists and the per-Gaussian fragment counts must equal the base frame's,
    # and the two one-sided differences must agree
    from paper_2503_01199_amd.raster import SceneTensors, Workspace, new_stats

    def loss_and_state(arrs):
        """Loss and the discrete state of the frame: every tile's depth-ordered list
        and every Gaussian's blended-fragment count (a change in any pixel's blended
        set changes some count)."""
        st = SceneTensors(*[torch.as_tensor(a, device=dev) for a in arrs], sc.sh_degree)
        fr = rz.forward(st, cams, workspace=Workspace(dev))
        loss = _loss64(fr.images, weights)
        ins = rz.inspect(fr)
        lists = torch.cat([ins["inst_tile"], ins["inst_record"]]).cpu()
        stats = new_stats(st.n, dev)
        rz.backward(fr, weights, stats=stats)
        return loss, (lists, stats["C"].cpu())

    arrays = [a.copy() for a in sc.arrays()]
    names = ("means", "log_scales", "quats", "opacity_logits", "sh")
    l0, s0 = loss_and_state(arrays)
    checked, tried = 0, 0
    while checked < 40 and tried < 400:
        tried += 1
        gi = int(rng.integers(0, 5))
        grad = g[gi].reshape(-1)
        idx = int(rng.choice(np.nonzero(np.abs(grad) > 1e-2 * np.abs(grad).max())[0]))
        x = np.float32(arrays[gi].reshape(-1)[idx])
        h = np.float32(max(abs(float(x)), 1e-1) * 3e-3)
        xp, xm = np.float32(x + h), np.float32(x - h)
        ap = [a.copy() for a in arrays]
        am = [a.copy() for a in arrays]
        ap[gi].reshape(-1)[idx] = xp
        am[gi].reshape(-1)[idx] = xm
        lp, sp = loss_and_state(ap)
        lm, sm = loss_and_state(am)
        if not all(a.shape == b.shape and torch.equal(a, b) for a, b in zip(sp + sm, s0 + s0)):
            continue
        # a rim pixel entering while another leaves keeps every count; the two
        # one-sided differences then disagree by the jump over h
        fp, fm = (lp - l0) / (float(xp) - float(x)), (l0 - lm) / (float(x) - float(xm))
        scale = max(abs(fp), abs(fm), 1e-2 * np.abs(grad).max())
        if abs(fp - fm) > 2e-2 * scale:
            continue
        fd = (lp - lm) / (float(xp) - float(xm))
        an = grad[idx]
        rel = abs(fd - an) / max(abs(an), 1e-2 * np.abs(grad).max())
        print("%-15s %6d fd %+.6g analytic %+.6g rel %.2g" % (names[gi], idx, fd, an, rel))
        assert rel < 2e-2
        checked += 1
    assert checked >= 30
