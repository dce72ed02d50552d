"""Packed-FP16 blend (Sec. 3.1.2) against the FP64 oracle, in both forms (alpha in
FP16; alpha and the forward's T in FP16): approximations whose error is reported,
not pinned.

G = 2^e and alpha = min(0.99, o G) run in FP16 (exponents rounded toward zero
from FP32); T, colour and the gradients stay FP32. The printed figures are the
error report (max abs, max relative with floor 1, normwise) per output. The
asserts are sanity bounds from the arithmetic, there to catch a broken kernel:
an exponent e in [-8, 0] rounded to FP16 is off by at most one unit in its last
place (2^-8 for |e| >= 4), so G, and with it alpha, is off by at most
ln(2) 2^-8 = 0.27 %, plus three FP16 roundings (3 x 2^-11 = 0.15 %). A pixel is a
T-weighted sum of alphas and colours, so its error stays below about 0.5 % of
its value; alphas within that margin of 1/255 may flip, each flip moving a pixel
by at most T alpha c < 0.005. Bounds: image normwise 5e-3, max abs 3e-2;
gradients normwise 5e-2 per parameter group (they carry the alpha error times
the colour-behind terms).
"""
import numpy as np
import pytest
import torch

import oracle as orc
from helpers import GRAD_TOL, IMAGE_TOL, ensure_built, grad_errors, image_errors, normwise
from paper_2503_01199_amd import scenes

pytestmark = pytest.mark.gpu

GROUPS = ("means", "log_scales", "quats", "opacity_logits", "sh")


@pytest.fixture(scope="module")
def rz():
    ensure_built()
    from paper_2503_01199_amd.raster import Rasterizer
    return Rasterizer(0)


def _forward(rz, scene, cams, precision):
    from paper_2503_01199_amd import _lib as L
    from paper_2503_01199_amd.raster import SceneTensors, Workspace
    prec = {"fp16": L.GSR_FP16_BLEND, "fp16t": L.GSR_FP16_BLEND_T}.get(precision, L.GSR_FP32)
    st = SceneTensors.from_scene(scene, rz.device)
    print("forward %s n=%d views=%s" % (precision, scene.n, [(c.width, c.height) for c in cams]), flush=True)
    fr = rz.forward(st, cams, precision=prec, workspace=Workspace(rz.device))
    torch.cuda.synchronize()
    return fr


def _image_report(img, ref, what):
    img = np.asarray(img, np.float64)
    ref = np.asarray(ref, np.float64)
    ab = np.abs(img - ref)
    rel = ab / np.maximum(1.0, np.abs(ref))
    nw = normwise(img, ref)
    print("%s: image max abs %.3g, max rel %.3g, normwise %.3g" % (what, ab.max(), rel.max(), nw))
    return float(ab.max()), nw


# sanity bounds per form (image normwise, image max abs, gradient normwise): the
# FP16-T form also rounds T to FP16 at every blend, a relative 2^-11 per blend that
# accumulates along a pixel's list
BOUNDS = {"fp16": (5e-3, 3e-2, 5e-2), "fp16t": (1e-2, 5e-2, 5e-2)}


@pytest.mark.parametrize("form", ["fp16", "fp16t"])
@pytest.mark.parametrize("which", ["tiny", "spheres"])
def test_fp16_blend_image_error(rz, which, form):
    if which == "tiny":
        sc, cam = scenes.tiny_scene(), scenes.tiny_camera()
    else:
        sc = scenes.spheres_planes_scene(60_000, seed_salt=2)
        cam = scenes.spheres_planes_camera()
    fr = _forward(rz, sc, [cam], form)
    ref = orc.render(sc, cam, mode=2)
    mx, nw = _image_report(fr.images[0].cpu().numpy(), ref["image"], "%s %s" % (form, which))
    assert nw < BOUNDS[form][0] and mx < BOUNDS[form][1]
    ins = rz.inspect(fr)
    T = ins["pixel_T"].cpu().numpy()
    assert (T >= 1e-4).all() and (T <= 1.0).all()
    # the integer stages do not depend on the blend precision
    f32 = _forward(rz, sc, [cam], "fp32")
    i32 = rz.inspect(f32)
    assert i32["info"]["instances"] == ins["info"]["instances"]
    assert torch.equal(i32["inst_record"], ins["inst_record"]) and torch.equal(i32["ranges"], ins["ranges"])


@pytest.mark.parametrize("form", ["fp16", "fp16t"])
def test_fp16_blend_gradient_error(rz, form):
    sc, cam = scenes.tiny_scene(), scenes.tiny_camera()
    ref = orc.render(sc, cam, mode=1)
    w, gt = scenes.l1_weights((3, cam.height, cam.width), config=0, salt=3)
    g = orc.l1_grad(ref["image"], w, gt).astype(np.float32)
    fr = _forward(rz, sc, [cam], form)
    grads = rz.backward(fr, [torch.as_tensor(g, device=rz.device)])
    torch.cuda.synchronize()
    ob = orc.backward(sc, cam, g.astype(np.float64), mode=1)
    for k in GROUPS:
        nw = normwise(grads[k].cpu().numpy(), ob[k])
        print("%s tiny gradient %s: normwise %.3g" % (form, k, nw))
        assert nw < BOUNDS[form][2], k


ROOM_WINDOW = (768, 832, 500, 564)


@pytest.fixture(scope="module")
def room_crop():
    """The 1M-Gaussian room at 1600x1064 (Morton order) with the loss restricted
    (weights 0 outside) to the 64x64 crop [768, 832) x [500, 564): the oracle's
    image and per-pixel state on the crop, the upstream gradient (zero outside the
    crop and on fragile pixels) and the oracle's backward for it."""
    sc, cam = scenes.room_scene(), scenes.room_camera()
    _, perm = orc.morton(sc.means)
    sc = sc.permuted(perm)
    win = ROOM_WINDOW
    ref = orc.render(sc, cam, mode=2, window=win, threads=8)
    w, gt = scenes.l1_weights((3, cam.height, cam.width), config=2)
    mask = np.zeros((cam.height, cam.width), bool)
    mask[win[2]:win[3], win[0]:win[1]] = True
    w = np.where(mask[None], w, 0.0).astype(np.float32)
    g = orc.l1_grad(ref["image"], w, gt).astype(np.float32)
    g[:, ~mask] = 0.0
    g[:, ref["fragile"]] = 0.0
    ob = orc.backward(sc, cam, g.astype(np.float64), mode=2, window=win, threads=8)
    return sc, cam, ref, g, ob


def _room_run(rz, room_crop, prec):
    from paper_2503_01199_amd.raster import SceneTensors, Workspace
    sc, cam, ref, g, ob = room_crop
    st = SceneTensors.from_scene(sc, rz.device)
    fr = rz.forward(st, [cam], precision=prec, workspace=Workspace(rz.device))
    grads = rz.backward(fr, [torch.as_tensor(g, device=rz.device)])
    torch.cuda.synchronize()
    win = ROOM_WINDOW
    crop = (slice(None), slice(win[2], win[3]), slice(win[0], win[1]))
    return fr, fr.images[0].cpu().numpy()[crop], {k: v.cpu().numpy() for k, v in grads.items()}, crop


def test_room_crop_fp32_matches_oracle(rz, room_crop):
    """FP32 path on the room crop at the parity bar: image and T per pixel within
    1e-5 on non-fragile pixels, the last blended position exact there, and every
    gradient element within 1e-3 (floor 1e-3 of the group's largest magnitude)
    on Gaussians no fragile pixel lists."""
    from paper_2503_01199_amd import _lib as L
    sc, cam, ref, g, ob = room_crop
    print("room crop fp32", flush=True)
    fr, img, grads, crop = _room_run(rz, room_crop, L.GSR_FP32)
    keep = ~ref["fragile"][crop[1:]]
    err, over, nfrag = image_errors(img, ref["image"][crop], ~keep)
    print("room crop fp32: image max rel %.3g over %d non-fragile pixels (%d fragile)" % (err, keep.sum(), nfrag))
    assert err <= IMAGE_TOL
    ins = rz.inspect(fr)
    T = ins["pixel_T"].cpu().numpy().reshape(cam.height, cam.width)[crop[1:]]
    last = ins["pixel_last"].cpu().numpy().view(np.uint32).reshape(cam.height, cam.width)[crop[1:]]
    eT = np.abs(T - ref["T"][crop[1:]])[keep].max()
    print("room crop fp32: T max abs %.3g; last blended position equal on %d of %d"
          % (eT, int((last == ref["n_contrib"][crop[1:]])[keep].sum()), int(keep.sum())))
    assert eT <= IMAGE_TOL
    assert np.array_equal(last[keep], ref["n_contrib"][crop[1:]][keep])
    skip = ob["fragile"]
    none = np.zeros_like(skip)
    for k in GROUPS:
        e_all = grad_errors(grads[k], ob[k], none)
        e = grad_errors(grads[k], ob[k], skip)
        print("room crop fp32 gradient %-15s max rel %.3g (every Gaussian %.3g), normwise %.3g"
              % (k, e, e_all, normwise(grads[k], ob[k])))
        assert e <= GRAD_TOL, k


@pytest.mark.parametrize("form", ["fp16", "fp16t"])
def test_fp16_blend_crop_of_the_room(rz, room_crop, form):
    """Error report of the FP16 blend (alpha in FP16; and with T in FP16 too) on the
    room crop against the oracle, with the sanity bounds of this module's header."""
    from paper_2503_01199_amd import _lib as L
    sc, cam, ref, g, ob = room_crop
    print("room crop %s" % form, flush=True)
    fr, img, grads, crop = _room_run(rz, room_crop, L.GSR_FP16_BLEND if form == "fp16" else L.GSR_FP16_BLEND_T)
    mx, nw = _image_report(img, ref["image"][crop], "room crop %s" % form)
    gn = {k: normwise(grads[k], ob[k]) for k in GROUPS}
    print("room crop %s gradient normwise: %s" % (form, ", ".join("%s %.3g" % kv for kv in gn.items())))
    b = BOUNDS[form]
    assert nw < b[0] and mx < b[1] and max(gn.values()) < b[2]
